// Batched MPCG in one persistent launch: every workgroup of kPB threads
// takes problems from a queue (largest first) and runs the whole of
// Algorithm 1 for one problem at a time.  Each step is a loop over that
// problem's nodes by the workgroup's threads with a barrier after it; the
// global reductions of the method (the Gram matrix and P^T r, W = Q^T Z,
// the residual norms) are workgroup reductions, and the step coefficients
// (pseudo-inverse, alpha, beta) and the stop decisions are made inside the
// workgroup with the same code as the single-block reduction kernels.  The
// problems are independent (the additive levels of one problem need no
// order among themselves, and different problems share nothing), so no
// synchronisation crosses workgroups and nothing is launched per step.
//
// Arithmetic per node is that of the batched step kernels (the same device
// helpers in the same order); the sums run over the workgroup's threads
// instead of over blocks, so results agree with the step-by-step path to
// rounding.
#pragma once

#include "batched.hpp"

namespace amg {

// Threads of a persistent workgroup: 8 waves, one workgroup per CU, so
// that each thread has 256 registers (the 6-column steps hold up to 37 FP64
// sums besides the node's loads).
#ifndef AMG_PB
#define AMG_PB 512
#endif
constexpr int kPB = AMG_PB;

// Nodes a thread works on at once in the steps over the finest level (the
// lighter steps, and those with wide per-node state): their results are
// formed in registers before any of them is stored, so the loads of all of
// them are in flight together (one workgroup per CU has few waves to hide
// memory latency with).  Each thread still visits its nodes in increasing
// order, so its sums are the same as node by node.  The loads of a group
// carry no branch: a node past the end is read at the last node (a valid
// address) and its operands are zeroed (they add exact zeros) or its stores
// skipped.
// The light steps take 8 nodes per thread at once (4 in 3D FP64), the wide
// ones 4 in 2D FP32, 2 in 2D FP64 and 3D FP32, 1 in 3D FP64: more would
// spill.
template <int DIM, typename T>
__host__ __device__ constexpr int pb_light() { return DIM == 3 && sizeof(T) == 8 ? 4 : 8; }
template <int DIM, typename T>
__host__ __device__ constexpr int pb_wide() {
    return DIM == 2 ? (sizeof(T) == 4 ? 4 : 2) : (sizeof(T) == 4 ? 2 : 1);
}

// Workgroup-shared state of the problem being solved.
struct PLds {
    double red[kMaxNB * (kMaxNB + 1) / 2 + kMaxNB];   // Gram upper triangle and P^T r
    double rw[1 + kMaxNB * kMaxNB];                   // ||r||^2 and W
    double G[kMaxNB * kMaxNB], Gp[kMaxNB * kMaxNB];
    double sab[kMaxNB + kMaxNB * kMaxNB];            // alpha and beta of the x/P update
    int state, zero_x, refresh, rank;
};

// Block carry up one level by the workgroup: Y_f[:, 0..NC-1] = P Y_c[:, 0..NC-1]
// (the arithmetic of prolong_at), kPU2 nodes per thread at once.
template <int DIM, typename T, int NC>
__device__ __forceinline__ void pb_prolong(const T* __restrict__ Yc, int nc, T* __restrict__ Yf, int nf, int Nf) {
    constexpr int SC = even_up(NC), SF = even_up(NC + 1);
    constexpr int kPU2 = pb_wide<DIM, T>();
    for (int base = threadIdx.x; base < Nf; base += kPB * kPU2) {
        T z[kPU2][SC];
#pragma unroll
        for (int u = 0; u < kPU2; ++u) {
            const int idx = min(base + u * kPB, Nf - 1);
            const Idx<DIM> p = decomp<DIM>(idx, nf);
            const XPar px = xparents(p.i, nc);
            const Par py = parents(p.j, nc);
            const Par pz = DIM == 3 ? parents(p.k, nc) : Par{0, 0, 1.f, 0.f, 1};
            interp_block<DIM, T, SC>(Yc, nc, px, py, pz, z[u]);
        }
#pragma unroll
        for (int u = 0; u < kPU2; ++u) {
            const int idx = base + u * kPB;
            if (idx < Nf) {
                T* o = Yf + (size_t)idx * SF;
#pragma unroll
                for (int c = 0; c < NC; ++c) o[c] = z[u][c];
            }
        }
    }
}

// Z = MG(r) of problem I by the workgroup: the finest smoother beside the
// restriction to level L-1 (both read r), then each restriction beside the
// smoother of the level it reads, the coarsest level's smoother, and the
// block carry up to level L-1; a barrier after every step.
template <int DIM, typename T>
__device__ __forceinline__ void pb_mg(const BInst<T>& I, T omega, int two) {
    constexpr int kPU = pb_light<DIM, T>();
    const int L = I.nlev - 1, nf = I.n[L], Nf = I.N[L];
    const int tid = threadIdx.x;
    for (int base = tid; base < Nf; base += kPB * kPU) {
        T c[kPU];
#pragma unroll
        for (int u = 0; u < kPU; ++u) {
            const int idx = min(base + u * kPB, Nf - 1);
            c[u] = fine_smooth_at<DIM, T, double>(I.op, I.r, idx, decomp<DIM>(idx, nf), omega, two);
        }
#pragma unroll
        for (int u = 0; u < kPU; ++u)
            if (base + u * kPB < Nf) I.cL[base + u * kPB] = c[u];
    }
    if (L > 0) {
        const int l = L - 1, Nl = I.N[l];
        const T* D = I.coef[l] + (size_t)stencil_center<DIM>() * Nl;
        for (int base = tid; base < Nl; base += kPB * kPU) {
            T g[kPU], d[kPU];
#pragma unroll
            for (int u = 0; u < kPU; ++u) {
                const int idx = min(base + u * kPB, Nl - 1);
                g[u] = restrict_at<DIM, double, T>(I.r, I.n[L], I.n[l], idx);
                d[u] = D[idx];
            }
#pragma unroll
            for (int u = 0; u < kPU; ++u) {
                const int idx = base + u * kPB;
                if (idx < Nl) {
                    I.g[l][idx] = g[u];
                    I.c1[l][idx] = omega * (g[u] / d[u]);
                }
            }
        }
    }
    __syncthreads();
    if (L == 0) return;
    // level m+1 is restricted: restrict it into m and smooth it
    for (int m = L - 2; m >= -1; --m) {
        if (m >= 0) {
            const int Nm = I.N[m];
            const T* D = I.coef[m] + (size_t)stencil_center<DIM>() * Nm;
            for (int base = tid; base < Nm; base += kPB * kPU) {
                T g[kPU], d[kPU];
#pragma unroll
                for (int u = 0; u < kPU; ++u) {
                    const int idx = min(base + u * kPB, Nm - 1);
                    g[u] = restrict_at<DIM, T, T>(I.g[m + 1], I.n[m + 1], I.n[m], idx);
                    d[u] = D[idx];
                }
#pragma unroll
                for (int u = 0; u < kPU; ++u) {
                    const int idx = base + u * kPB;
                    if (idx < Nm) {
                        I.g[m][idx] = g[u];
                        I.c1[m][idx] = omega * (g[u] / d[u]);
                    }
                }
            }
        }
        const int s = m + 1, Ns = I.N[s];
        const CoarseOp<T> op{I.n[s], Ns, I.coef[s], 0};
        for (int base = tid; base < Ns; base += kPB * kPU) {
            T c[kPU];
#pragma unroll
            for (int u = 0; u < kPU; ++u)
                c[u] = coarse_smooth_at<DIM, T>(op, I.g[s], I.c1[s], nullptr, min(base + u * kPB, Ns - 1), omega, 0,
                                                two);
#pragma unroll
            for (int u = 0; u < kPU; ++u)
                if (base + u * kPB < Ns) I.Y[s][(size_t)(base + u * kPB) * even_up(s + 1) + s] = c[u];
        }
        __syncthreads();
    }
    // block carry Y_{l+1}[:, 0..l] = P Y_l, l = 0 .. L-2
    for (int l = 0; l + 1 < L; ++l) {
        switch (l + 1) {
            case 1: pb_prolong<DIM, T, 1>(I.Y[l], I.n[l], I.Y[l + 1], I.n[l + 1], I.N[l + 1]); break;
            case 2: pb_prolong<DIM, T, 2>(I.Y[l], I.n[l], I.Y[l + 1], I.n[l + 1], I.N[l + 1]); break;
            case 3: pb_prolong<DIM, T, 3>(I.Y[l], I.n[l], I.Y[l + 1], I.n[l + 1], I.N[l + 1]); break;
            default: pb_prolong<DIM, T, 4>(I.Y[l], I.n[l], I.Y[l + 1], I.n[l + 1], I.N[l + 1]); break;
        }
        __syncthreads();
    }
}

// The directions at fine node idx: the coarse corrections interpolated from
// the level-(L-1) block carry and the finest smoother output.
template <int DIM, typename T, int NB>
__device__ __forceinline__ void pb_z(const BInst<T>& I, int idx, const Idx<DIM>& p, T (&z)[NB]) {
    const int L = I.nlev - 1;
    fine_z<DIM, T, NB, 0>(L > 0 ? I.Y[L - 1] : nullptr, L > 0 ? I.n[L - 1] : 1, I.cL, nullptr, false, idx, p, z);
}

// Q = A P, the Gram upper triangle and P^T r, then the alpha step
// (pseudo-inverse, alpha = G^+ P^T r, breakdown), by the workgroup.
template <int DIM, typename T, int NB>
__device__ __forceinline__ void pb_spmm_alpha(const BInst<T>& I, PLds& sh) {
    constexpr int NG = NB * (NB + 1) / 2;
    constexpr int S = even_up(NB);
    constexpr int kPU2 = pb_wide<DIM, T>();
    const int L = I.nlev - 1, n = I.n[L], N = I.N[L];
    double acc[NG + NB];
#pragma unroll
    for (int q = 0; q < NG + NB; ++q) acc[q] = 0.0;
    for (int base = threadIdx.x; base < N; base += kPB * kPU2) {
        T pv[kPU2][S], qv[kPU2][S];
        double ri[kPU2];
#pragma unroll
        for (int u = 0; u < kPU2; ++u) {
            const int idx = min(base + u * kPB, N - 1);
            fine_apply_block<DIM, T, S>(I.op, I.P, idx, decomp<DIM>(idx, n), pv[u], qv[u]);
            ri[u] = I.r[idx];
        }
#pragma unroll
        for (int u = 0; u < kPU2; ++u) {
            const int idx = base + u * kPB;
            if (idx >= N) continue;
            store_node<T, S>(I.Q + (size_t)idx * S, qv[u]);
            int q = 0;
#pragma unroll
            for (int a = 0; a < NB; ++a)
#pragma unroll
                for (int c = a; c < NB; ++c) acc[q++] += double(pv[u][a]) * double(qv[u][c]);
#pragma unroll
            for (int a = 0; a < NB; ++a) acc[NG + a] += double(pv[u][a]) * ri[u];
        }
    }
    block_reduce_bs<NG + NB, kPB>(acc, sh.red);
    alpha_apply<NB>(I.ctl, sh.red, sh.G, sh.Gp, &sh.rank, I.small + kMaxNB + kMaxNB * kMaxNB, I.small, nullptr);
    __syncthreads();
    if (threadIdx.x == 0) sh.state = I.ctl->state;
    __syncthreads();
}

// x += P alpha (deferred update of Algorithm 1), and unless stopping
// (state 1), P = Z - P beta in place; init: P_0 = Z_0 only.
template <int DIM, typename T, int NB>
__device__ __forceinline__ void pb_update_xP(const BInst<T>& I, PLds& sh, int init, int state) {
    constexpr int S = even_up(NB);
    constexpr int kPU2 = pb_wide<DIM, T>();
    const int L = I.nlev - 1, n = I.n[L], N = I.N[L];
    const bool newP = init || state == 0;
    for (int base = threadIdx.x; base < N; base += kPB * kPU2) {
        T pk[kPU2][S], z[kPU2][NB];
        double xi[kPU2];
#pragma unroll
        for (int u = 0; u < kPU2; ++u) {
            const int idx = min(base + u * kPB, N - 1);
#pragma unroll
            for (int c = 0; c < S; ++c) pk[u][c] = T(0);
#pragma unroll
            for (int c = 0; c < NB; ++c) z[u][c] = T(0);
            xi[u] = 0.0;
            if (!init) {
                load_node<T, S>(I.P + (size_t)idx * S, pk[u]);
                xi[u] = I.x[idx];
            }
            if (newP) pb_z<DIM, T, NB>(I, idx, decomp<DIM>(idx, n), z[u]);
        }
#pragma unroll
        for (int u = 0; u < kPU2; ++u) {
            const int idx = base + u * kPB;
            if (idx >= N) continue;
            if (!init) {
                double v = xi[u];
#pragma unroll
                for (int c = 0; c < NB; ++c) v += double(pk[u][c]) * sh.sab[c];
                I.x[idx] = v;
            }
            if (!newP) continue;
            T pn[S];
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                double v = double(z[u][c]);
                if (!init) {
#pragma unroll
                    for (int a2 = 0; a2 < NB; ++a2) v -= double(pk[u][a2]) * sh.sab[NB + a2 * NB + c];
                }
                pn[c] = T(v);
            }
#pragma unroll
            for (int c = NB; c < S; ++c) pn[c] = T(0);
            store_node<T, S>(I.P + (size_t)idx * S, pn);
        }
    }
    __syncthreads();
}

// Algorithm 1 for problem I by the whole workgroup, until it stops
// (converged, maxit, breakdown or non-finite); the problem's control word
// holds the tolerance on entry and the outcome on return.
template <int DIM, typename T, int NB>
__device__ void pb_solve(const BInst<T>& I, T omega, int two, int mixed, PLds& sh) {
    constexpr int kPU = pb_light<DIM, T>();
    static_assert(1 + NB * NB <= 40, "the W reduction runs in one group of values");
    constexpr int kPU2 = pb_wide<DIM, T>();
    const int L = I.nlev - 1, n = I.n[L], N = I.N[L];
    const int tid = threadIdx.x;
    Ctl* ctl = I.ctl;
    // r_0 = b - A x_0 (FP64), ||b||^2 and ||r_0||^2
    {
        double v[2] = {0.0, 0.0};
        for (int base = tid; base < N; base += kPB * kPU) {
            double bi[kPU], ri[kPU];
#pragma unroll
            for (int u = 0; u < kPU; ++u) {
                const int idx = min(base + u * kPB, N - 1);
                bi[u] = I.b[idx];
                ri[u] = bi[u] - fine_apply<DIM, double>(I.op64, I.x, idx, decomp<DIM>(idx, n));
            }
#pragma unroll
            for (int u = 0; u < kPU; ++u) {
                const int idx = base + u * kPB;
                if (idx >= N) continue;
                I.r[idx] = ri[u];
                v[0] += bi[u] * bi[u];
                v[1] += ri[u] * ri[u];
            }
        }
        block_reduce_bs<2, kPB>(v, sh.red);
        if (tid == 0) {
            init_decide(ctl, sh.red[0], sh.red[1], ctl->tol, nullptr);
            sh.state = ctl->state;
            sh.zero_x = ctl->zero_x;
        }
        __syncthreads();
    }
    if (sh.zero_x)
        for (int idx = tid; idx < N; idx += kPB) I.x[idx] = 0.0;
    if (sh.state != 0) return;
    // Z_0, P_0 = Z_0, Q_0 = A P_0 and alpha_0
    pb_mg<DIM, T>(I, omega, two);
    pb_update_xP<DIM, T, NB>(I, sh, 1, 0);
    pb_spmm_alpha<DIM, T, NB>(I, sh);
    const int maxit = ctl->maxit;
    for (int k = 0; k <= maxit + 1; ++k) {
        if (sh.state == 2) break;
        // r_{k+1} = r_k - Q_k alpha_k, ||r_{k+1}||^2 kept for the beta step
        double w[1 + NB * NB];
#pragma unroll
        for (int q = 0; q < 1 + NB * NB; ++q) w[q] = 0.0;
        {
            constexpr int S = even_up(NB);
            double a[NB];
#pragma unroll
            for (int c = 0; c < NB; ++c) a[c] = I.small[c];
            for (int base = tid; base < N; base += kPB * kPU) {
                T q[kPU][S];
                double ri[kPU];
#pragma unroll
                for (int u = 0; u < kPU; ++u) {
                    const int idx = min(base + u * kPB, N - 1);
                    load_node<T, S>(I.Q + (size_t)idx * S, q[u]);
                    ri[u] = I.r[idx];
                }
#pragma unroll
                for (int u = 0; u < kPU; ++u) {
                    const int idx = base + u * kPB;
                    if (idx >= N) continue;
                    double v = ri[u];
#pragma unroll
                    for (int c = 0; c < NB; ++c) v -= double(q[u][c]) * a[c];
                    I.r[idx] = v;
                    w[0] += v * v;
                }
            }
            __syncthreads();
        }
        // Z_{k+1} = MG(r_{k+1}) and W = Q_k^T Z_{k+1}
        pb_mg<DIM, T>(I, omega, two);
        {
            constexpr int S = even_up(NB);
            for (int base = tid; base < N; base += kPB * kPU2) {
                T z[kPU2][NB], q[kPU2][S];
#pragma unroll
                for (int u = 0; u < kPU2; ++u) {
                    const int idx = min(base + u * kPB, N - 1);
                    pb_z<DIM, T, NB>(I, idx, decomp<DIM>(idx, n), z[u]);
                    load_node<T, S>(I.Q + (size_t)idx * S, q[u]);
                }
#pragma unroll
                for (int u = 0; u < kPU2; ++u) {
                    if (base + u * kPB >= N) continue;
#pragma unroll
                    for (int a = 0; a < NB; ++a) {
                        const double qa = double(q[u][a]);
#pragma unroll
                        for (int c = 0; c < NB; ++c) w[1 + a * NB + c] += qa * double(z[u][c]);
                    }
                }
            }
        }
        block_reduce_bs<1 + NB * NB, kPB>(w, sh.rw);
        // residual check, beta = G_k^+ W
        if (tid == 0) sh.state = beta_decide(ctl, sh.rw[0], nullptr, mixed);
        __syncthreads();
        const int st = sh.state;
        if (st == 0) beta_apply<NB>(I.small + kMaxNB + kMaxNB * kMaxNB, sh.rw + 1, I.small + kMaxNB, tid, kPB);
        __syncthreads();
        for (int q = tid; q < NB + NB * NB; q += kPB) sh.sab[q] = q < NB ? I.small[q] : I.small[kMaxNB + q - NB];
        __syncthreads();
        // x_{k+1} = x_k + P_k alpha_k; P_{k+1} = Z_{k+1} - P_k beta
        pb_update_xP<DIM, T, NB>(I, sh, 0, st);
        // FP32 bulk: the true residual replaces r when requested
        if (mixed) {
            if (tid == 0) sh.refresh = ctl->refresh_req;
            __syncthreads();
            if (sh.refresh) {
                double v[1] = {0.0};
                for (int base = tid; base < N; base += kPB * kPU) {
                    double ri[kPU];
#pragma unroll
                    for (int u = 0; u < kPU; ++u) {
                        const int idx = min(base + u * kPB, N - 1);
                        ri[u] = I.b[idx] - fine_apply<DIM, double>(I.op64, I.x, idx, decomp<DIM>(idx, n));
                    }
#pragma unroll
                    for (int u = 0; u < kPU; ++u) {
                        const int idx = base + u * kPB;
                        if (idx >= N) continue;
                        I.r[idx] = ri[u];
                        v[0] += ri[u] * ri[u];
                    }
                }
                block_reduce_bs<1, kPB>(v, sh.red);
                if (tid == 0) {
                    refresh_decide(ctl, sh.red[0], nullptr);
                    sh.state = ctl->state;
                }
                __syncthreads();
            }
        }
        // Q_{k+1} = A P_{k+1}, Gram, alpha_{k+1}; a stop after the x update ends here
        if (sh.state == 0) {
            pb_spmm_alpha<DIM, T, NB>(I, sh);
        } else if (sh.state == 1) {
            __syncthreads();
            if (tid == 0) {
                ctl->state = 2;
                sh.state = 2;
            }
            __syncthreads();
        }
    }
}

// The persistent launch: workgroups take problems order[0], order[1], ...
// from the queue counter (zero on entry) until every problem is taken.
template <int DIM, typename T>
__global__ void __launch_bounds__(kPB, 1) k_b_persistent(const BInst<T>* __restrict__ insts,
                                                        const int* __restrict__ order, int count, int* queue,
                                                        T omega, int two, int mixed) {
    __shared__ PLds sh;
    __shared__ int qs;
    for (int round = 0; round < count; ++round) {
        if (threadIdx.x == 0) qs = atomicAdd(queue, 1);
        __syncthreads();
        // the problem index is uniform: read it into a scalar register, so
        // that the instance's fields come in by scalar loads
        const int q = __builtin_amdgcn_readfirstlane(qs);
        __syncthreads();
        if (q >= count) return;
        const BInst<T>& I = insts[__builtin_amdgcn_readfirstlane(order[q])];
        switch (I.nlev) {
            case 1: pb_solve<DIM, T, 1>(I, omega, two, mixed, sh); break;
            case 2: pb_solve<DIM, T, 2>(I, omega, two, mixed, sh); break;
            case 3: pb_solve<DIM, T, 3>(I, omega, two, mixed, sh); break;
            case 4: pb_solve<DIM, T, 4>(I, omega, two, mixed, sh); break;
            case 5: pb_solve<DIM, T, 5>(I, omega, two, mixed, sh); break;
            default: pb_solve<DIM, T, 6>(I, omega, two, mixed, sh); break;
        }
        __syncthreads();
    }
}

// The queue counter of the next persistent launch (a plain store, so that
// the reset can sit in a captured graph).
static __global__ void k_b_reset_queue(int* queue) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *queue = 0;
}

}  // namespace amg
