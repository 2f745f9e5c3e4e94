// Batched persistent MPCG: many independent structured problems (each with
// its own grid size, hierarchy and right-hand side) solved by one kernel
// launch.  Workgroups pull instances, largest first, from an atomic queue;
// one 1024-thread workgroup runs the whole of Algorithm 1 for an instance,
// every phase a loop over that instance's nodes followed by a workgroup
// barrier, reductions in a fixed order through LDS.  No workgroup ever waits
// for another, and every workgroup exits once the queue is drained.
#pragma once

#include "common.hpp"
#include "grid_kernels.hpp"
#include "small_kernels.hpp"

namespace amg {

constexpr int kBatchBlock = 1024;
constexpr int kBatchWaves = kBatchBlock / 64;

template <typename T>
struct BInst {
    int nlev;                      // levels; search directions NB = nlev
    int n[kMaxLevels];             // nodes per axis, 0 = coarsest
    int N[kMaxLevels];
    const T* coef[kMaxLevels];     // coarse levels: 3^d stencil coefficients
    T* g[kMaxLevels];              // restricted residual
    T* c1[kMaxLevels];             // first Jacobi sweep
    T* Y[kMaxLevels];              // node-major block carry
    const double* b;
    double* x;
    double* r;
    T* P;                          // node-major, stride even_up(NB)
    T* Q;
    T* cL;
};

struct BOut {
    int status, iterations, refreshes, rank;
    double bnorm, relres;
};

struct BatchParams {
    int count;
    const int* order;      // instance indices, largest first
    int* queue;            // next position in order (reset to 0 before each launch)
    double tol;
    int maxit;
    int two_sweeps;
    double omega;
    double tau;            // eigenvalue cut; <= 0: 64 * NB * unit for each problem
    double unit;           // unit roundoff of the bulk type
    double drop2;          // mixed form: refresh when ||r||^2 fell by this factor
    int mixed;
    BOut* out;
};

// Sum K per-thread values over the 1024-thread workgroup into res[k]
// (shared); scratch: shared [kBatchWaves][64] doubles.  v is destroyed.
template <int K>
__device__ __forceinline__ void batch_reduce(double (&v)[K], double* res, double* scratch) {
    constexpr int KP = pow2_up(K);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int vi = wave_reduce_multi<K>(v);
    if ((lane & (64 / KP - 1)) == 0) scratch[w * 64 + vi] = v[0];
    __syncthreads();
    if (threadIdx.x < K) {
        double s = scratch[threadIdx.x];
        for (int q = 1; q < kBatchWaves; ++q) s += scratch[q * 64 + threadIdx.x];
        res[threadIdx.x] = s;
    }
    __syncthreads();
}

template <int NB>
struct BShared {
    double red[64];
    double G[NB * NB];
    double Gp[NB * NB];
    double alpha[NB];
    double beta[NB * NB];
    int rank;
};

// Z = MG(r): fine smoother, restriction chain, all coarse levels smoothed,
// prolongation chain; barriers between dependent phases.
template <int DIM, typename T, int NB>
__device__ void batch_mg(const BInst<T>& I, const FineOp<T>& op, const double* __restrict__ r, T omega,
                         int two) {
    constexpr int L = NB - 1;
    const int N = I.N[L];
    for (int idx = threadIdx.x; idx < N; idx += kBatchBlock) {
        const Idx<DIM> p = decomp<DIM>(idx, op.n);
        I.cL[idx] = fine_smooth_at<DIM, T, double>(op, r, idx, p, omega, two);
    }
    if (L == 0) {
        __syncthreads();
        return;
    }
    {
        const int m = L - 1;
        const T* D = I.coef[m] + (size_t)stencil_center<DIM>() * I.N[m];
        for (int idx = threadIdx.x; idx < I.N[m]; idx += kBatchBlock) {
            const T g = restrict_at<DIM, double, T>(r, I.n[L], I.n[m], idx);
            I.g[m][idx] = g;
            I.c1[m][idx] = omega * (g / D[idx]);
        }
        __syncthreads();
    }
    for (int m = L - 2; m >= 0; --m) {
        const T* D = I.coef[m] + (size_t)stencil_center<DIM>() * I.N[m];
        for (int idx = threadIdx.x; idx < I.N[m]; idx += kBatchBlock) {
            const T g = restrict_at<DIM, T, T>(I.g[m + 1], I.n[m + 1], I.n[m], idx);
            I.g[m][idx] = g;
            I.c1[m][idx] = omega * (g / D[idx]);
        }
        __syncthreads();
    }
    for (int l = 0; l < L; ++l) {
        CoarseOp<T> cop{I.n[l], I.N[l], I.coef[l]};
        const int S = even_up(l + 1);
        for (int idx = threadIdx.x; idx < I.N[l]; idx += kBatchBlock)
            I.Y[l][(size_t)idx * S + l] = coarse_smooth_at<DIM, T>(cop, I.g[l], I.c1[l], nullptr, idx, omega, 0, two);
    }
    __syncthreads();
    for (int l = 0; l + 1 < L; ++l) {
        for (int idx = threadIdx.x; idx < I.N[l + 1]; idx += kBatchBlock) {
            switch (l + 1) {
                case 1: prolong_at<DIM, T, 1>(I.Y[l], I.n[l], I.Y[l + 1], I.n[l + 1], idx); break;
                case 2: prolong_at<DIM, T, 2>(I.Y[l], I.n[l], I.Y[l + 1], I.n[l + 1], idx); break;
                case 3: prolong_at<DIM, T, 3>(I.Y[l], I.n[l], I.Y[l + 1], I.n[l + 1], idx); break;
                case 4: prolong_at<DIM, T, 4>(I.Y[l], I.n[l], I.Y[l + 1], I.n[l + 1], idx); break;
                case 5: prolong_at<DIM, T, 5>(I.Y[l], I.n[l], I.Y[l + 1], I.n[l + 1], idx); break;
                default: prolong_at<DIM, T, 6>(I.Y[l], I.n[l], I.Y[l + 1], I.n[l + 1], idx); break;
            }
        }
        __syncthreads();
    }
}

// Q = A P, Gram and g = P^T r, pseudo-inverse, alpha (into shared state).
template <int DIM, typename T, int NB>
__device__ void batch_gram_alpha(const BInst<T>& I, const FineOp<T>& op, BShared<NB>& sh, double tau,
                                 double* scratch) {
    constexpr int NG = NB * (NB + 1) / 2, S = even_up(NB);
    constexpr int L = NB - 1;
    const int N = I.N[L];
    double acc[NG + NB];
#pragma unroll
    for (int q = 0; q < NG + NB; ++q) acc[q] = 0.0;
    for (int idx = threadIdx.x; idx < N; idx += kBatchBlock) {
        const Idx<DIM> p = decomp<DIM>(idx, op.n);
        T pv[S], qv[S];
        fine_apply_block<DIM, T, S>(op, I.P, idx, p, pv, qv);
        store_node<T, S>(I.Q + (size_t)idx * S, qv);
        const double ri = I.r[idx];
        int q = 0;
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int c = a; c < NB; ++c) acc[q++] += double(pv[a]) * double(qv[c]);
#pragma unroll
        for (int a = 0; a < NB; ++a) acc[NG + a] += double(pv[a]) * ri;
    }
    batch_reduce<NG + NB>(acc, sh.red, scratch);
    if (threadIdx.x == 0) {
        int q = 0;
        for (int a = 0; a < NB; ++a)
            for (int c = a; c < NB; ++c, ++q) sh.G[a * NB + c] = sh.G[c * NB + a] = sh.red[q];
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        const int rk = wave_pinv<NB>(sh.G, tau, sh.Gp);
        if (threadIdx.x == 0) sh.rank = rk;
    }
    __syncthreads();
    if (threadIdx.x < NB) {
        double s = 0.0;
        for (int m = 0; m < NB; ++m) s += sh.Gp[threadIdx.x * NB + m] * sh.red[NG + m];
        sh.alpha[threadIdx.x] = s;
    }
    __syncthreads();
}

// ||r||^2 after r = b - A x in FP64 (start and refreshes).
template <int DIM>
__device__ void batch_residual(const FineOp<double>& op64, const double* __restrict__ b,
                               const double* __restrict__ x, double* __restrict__ r, double* res2 /*shared 2*/,
                               double* scratch) {
    double acc[2] = {0.0, 0.0};
    for (int idx = threadIdx.x; idx < op64.N; idx += kBatchBlock) {
        const Idx<DIM> p = decomp<DIM>(idx, op64.n);
        const double bi = b[idx];
        const double ri = bi - fine_apply<DIM, double>(op64, x, idx, p);
        r[idx] = ri;
        acc[0] += bi * bi;
        acc[1] += ri * ri;
    }
    batch_reduce<2>(acc, res2, scratch);
}

template <int DIM, typename T, int NB>
__device__ void solve_instance(const BInst<T>& I, const BatchParams& bp, BOut& out, double* scratch) {
    constexpr int L = NB - 1, S = even_up(NB);
    __shared__ BShared<NB> sh;
    const int nf = I.n[L], N = I.N[L];
    const double h2inv = double(nf + 1) * double(nf + 1);
    FineOp<T> op{nf, N, T(h2inv), nullptr, nullptr, nullptr, nullptr, T(1.0 / (2 * DIM * h2inv)), nullptr};
    FineOp<double> op64{nf, N, h2inv, nullptr, nullptr, nullptr, nullptr, 1.0 / (2 * DIM * h2inv), nullptr};
    const T omega = T(bp.omega);
    const int nc = L > 0 ? I.n[L - 1] : 1;
    const T* Ytop = L > 0 ? I.Y[L - 1] : nullptr;
    const double tau = bp.tau > 0 ? bp.tau : 64.0 * NB * bp.unit;

    batch_residual<DIM>(op64, I.b, I.x, I.r, sh.red, scratch);
    const double bn2 = sh.red[0];
    double rho = sh.red[1];
    int status = kOK, it = 0, refreshes = 0;
    const double tol2 = bp.tol * bp.tol * bn2;
    if (bn2 == 0.0) {
        for (int idx = threadIdx.x; idx < N; idx += kBatchBlock) I.x[idx] = 0.0;
        rho = 0.0;
    } else if (!isfinite(rho) || !isfinite(bn2)) {
        status = kNONFINITE;
    } else if (!(rho <= tol2)) {
        batch_mg<DIM, T, NB>(I, op, I.r, omega, bp.two_sweeps);
        for (int idx = threadIdx.x; idx < N; idx += kBatchBlock) {
            const Idx<DIM> p = decomp<DIM>(idx, nf);
            T z[NB], pn[S];
            fine_z<DIM, T, NB, 0>(Ytop, nc, I.cL, nullptr, false, idx, p, z);
#pragma unroll
            for (int c = 0; c < S; ++c) pn[c] = c < NB ? z[c] : T(0);
            store_node<T, S>(I.P + (size_t)idx * S, pn);
        }
        __syncthreads();
        batch_gram_alpha<DIM, T, NB>(I, op, sh, tau, scratch);
        double rho_ref = rho;
        while (true) {
            if (sh.rank == 0) {
                status = kBREAKDOWN;
                break;
            }
            // r_{k+1} = r_k - Q alpha, ||r||^2
            double a1[1] = {0.0};
            for (int idx = threadIdx.x; idx < N; idx += kBatchBlock) {
                T q[S];
                load_node<T, S>(I.Q + (size_t)idx * S, q);
                double ri = I.r[idx];
#pragma unroll
                for (int c = 0; c < NB; ++c) ri -= double(q[c]) * sh.alpha[c];
                I.r[idx] = ri;
                a1[0] += ri * ri;
            }
            batch_reduce<1>(a1, sh.red, scratch);
            rho = sh.red[0];
            ++it;
            int stop = 0, refresh = 0;
            if (!isfinite(rho)) {
                status = kNONFINITE;
                stop = 1;
            } else if (rho <= tol2 && !bp.mixed) {
                stop = 1;
            } else if (it >= bp.maxit) {
                status = kMAXIT;
                stop = 1;
            } else if (bp.mixed && (rho <= tol2 || rho <= bp.drop2 * rho_ref)) {
                refresh = 1;
            }
            if (stop) {
                for (int idx = threadIdx.x; idx < N; idx += kBatchBlock) {
                    T pk[S];
                    load_node<T, S>(I.P + (size_t)idx * S, pk);
                    double xi = I.x[idx];
#pragma unroll
                    for (int c = 0; c < NB; ++c) xi += double(pk[c]) * sh.alpha[c];
                    I.x[idx] = xi;
                }
                break;
            }
            batch_mg<DIM, T, NB>(I, op, I.r, omega, bp.two_sweeps);
            // W = Q^T Z, beta = G^+ W
            {
                double w[NB * NB];
#pragma unroll
                for (int q = 0; q < NB * NB; ++q) w[q] = 0.0;
                for (int idx = threadIdx.x; idx < N; idx += kBatchBlock) {
                    const Idx<DIM> p = decomp<DIM>(idx, nf);
                    T z[NB], q[S];
                    fine_z<DIM, T, NB, 0>(Ytop, nc, I.cL, nullptr, false, idx, p, z);
                    load_node<T, S>(I.Q + (size_t)idx * S, q);
#pragma unroll
                    for (int a = 0; a < NB; ++a)
#pragma unroll
                        for (int c = 0; c < NB; ++c) w[a * NB + c] += double(q[a]) * double(z[c]);
                }
                batch_reduce<NB * NB>(w, sh.red, scratch);
                if (threadIdx.x < NB * NB) {
                    const int a = threadIdx.x / NB, c = threadIdx.x % NB;
                    double s = 0.0;
                    for (int m = 0; m < NB; ++m) s += sh.Gp[a * NB + m] * sh.red[m * NB + c];
                    sh.beta[threadIdx.x] = s;
                }
                __syncthreads();
            }
            // x += P_k alpha_k;  P_{k+1} = Z - P_k beta
            for (int idx = threadIdx.x; idx < N; idx += kBatchBlock) {
                const Idx<DIM> p = decomp<DIM>(idx, nf);
                T pk[S], z[NB], pn[S];
                load_node<T, S>(I.P + (size_t)idx * S, pk);
                double xi = I.x[idx];
#pragma unroll
                for (int c = 0; c < NB; ++c) xi += double(pk[c]) * sh.alpha[c];
                I.x[idx] = xi;
                fine_z<DIM, T, NB, 0>(Ytop, nc, I.cL, nullptr, false, idx, p, z);
#pragma unroll
                for (int c = 0; c < S; ++c) {
                    if (c < NB) {
                        double v = double(z[c]);
#pragma unroll
                        for (int a = 0; a < NB; ++a) v -= double(pk[a]) * sh.beta[a * NB + c];
                        pn[c] = T(v);
                    } else {
                        pn[c] = T(0);
                    }
                }
                store_node<T, S>(I.P + (size_t)idx * S, pn);
            }
            __syncthreads();
            if (refresh) {
                batch_residual<DIM>(op64, I.b, I.x, I.r, sh.red, scratch);
                rho = sh.red[1];
                rho_ref = rho;
                ++refreshes;
                if (!isfinite(rho)) {
                    status = kNONFINITE;
                    break;
                }
                if (rho <= tol2) break;
            }
            batch_gram_alpha<DIM, T, NB>(I, op, sh, tau, scratch);
        }
    }
    if (threadIdx.x == 0) {
        out.status = status;
        out.iterations = it;
        out.refreshes = refreshes;
        out.rank = sh.rank;
        out.bnorm = sqrt(bn2);
        out.relres = bn2 > 0 ? sqrt(rho / bn2) : 0.0;
    }
    __syncthreads();
}

__global__ void k_queue_reset(int* queue) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *queue = 0;
}

template <int DIM, typename T>
__global__ void __launch_bounds__(kBatchBlock) k_batched(const BInst<T>* __restrict__ insts,
                                                         const BatchParams* __restrict__ bpp) {
    __shared__ double scratch[kBatchWaves * 64];
    __shared__ int slot;
    const BatchParams bp = *bpp;
    while (true) {
        if (threadIdx.x == 0) slot = atomicAdd(bp.queue, 1);
        __syncthreads();
        const int q = slot;
        __syncthreads();
        if (q >= bp.count) break;
        const int id = bp.order[q];
        const BInst<T>& I = insts[id];
        switch (I.nlev) {
            case 1: solve_instance<DIM, T, 1>(I, bp, bp.out[id], scratch); break;
            case 2: solve_instance<DIM, T, 2>(I, bp, bp.out[id], scratch); break;
            case 3: solve_instance<DIM, T, 3>(I, bp, bp.out[id], scratch); break;
            case 4: solve_instance<DIM, T, 4>(I, bp, bp.out[id], scratch); break;
            case 5: solve_instance<DIM, T, 5>(I, bp, bp.out[id], scratch); break;
            default: solve_instance<DIM, T, 6>(I, bp, bp.out[id], scratch); break;
        }
    }
}

}  // namespace amg
