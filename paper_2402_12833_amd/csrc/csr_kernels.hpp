// Kernels of one MPCG iteration (Algorithm 1) for a general hierarchy given
// as sparse matrices: the fine operator A, the prolongations P_l (level l
// to l+1) and the restrictions R_l = s P_l^T, all in CSR (int32 row
// pointers and column indices, values in the bulk type T; the fine operator
// also in FP64 for r = b - A x).  Coarse operators are the Galerkin products
// built on the host.  One thread per row, grid-stride over the rows; the
// direction blocks are node-major as in the structured path.  The
// reductions and the residual update are the structured path's.
#pragma once

#include "common.hpp"
#include "grid_kernels.hpp"

namespace amg {

// A sparse matrix given in CSR, stored on the device sliced: slices of 64
// consecutive rows (one wavefront), each padded to its longest row and
// stored column by column (entry k of row 64 s + l at soff[s] + 64 k + l),
// so that the 64 lanes of a wave read 64 consecutive entries per step and
// loop the same number of times.  A row's stored entries come in its CSR
// order, then padding of weight 0 at one of the row's own columns, so every
// row sum is the CSR one plus exact zeros.
template <typename T>
struct CsrOp {
    int n;              // rows
    const int* soff;    // per slice: first entry
    const int* swid;    // per slice: entries per row (padded)
    const int* col;
    const T* val;
};

// f(column, value) for the stored entries of row i in order.  The rows of a
// wave must be the 64 rows of one slice (loops start waves at multiples of
// 64), so soff and swid are wave-uniform.
// Entries are taken in groups of four: the group's column indices and
// weights are loaded together before f runs on them in row order, so the
// gathers f makes through them do not wait on one index load each.  The
// order in which f sees the entries is the row order either way.
constexpr int kRowGroup = 4;   // eight measured slower (more registers held per lane)

template <typename T, typename F>
__device__ __forceinline__ void for_row(const CsrOp<T>& A, int i, F&& f) {
    const int s = i >> 6;
    const int off = A.soff[s] + (i & 63), w = A.swid[s];
    int k = 0;
    for (; k + kRowGroup <= w; k += kRowGroup) {
        int c[kRowGroup];
        T v[kRowGroup];
#pragma unroll
        for (int u = 0; u < kRowGroup; ++u) {
            c[u] = A.col[off + 64 * (k + u)];
            v[u] = A.val[off + 64 * (k + u)];
        }
#pragma unroll
        for (int u = 0; u < kRowGroup; ++u) f(c[u], v[u]);
    }
    for (; k < w; ++k) f(A.col[off + 64 * k], A.val[off + 64 * k]);
}

template <typename C, typename T, typename F>
__device__ __forceinline__ C csr_row_dot(const CsrOp<T>& A, int i, F&& u) {
    C acc = C(0);
    for_row(A, i, [&](int j, T v) { acc += C(v) * C(u(j)); });
    return acc;
}

#define CSR_LOOP(i, n) for (int i = blockIdx.x * kBlock + threadIdx.x; i < (n); i += gridDim.x * kBlock)

// r = b - A x (FP64), partial ||b||^2 and ||r||^2.
static __global__ void __launch_bounds__(kBlock) k_csr_init_residual(CsrOp<double> A, const double* __restrict__ b,
                                                              const double* __restrict__ x, double* __restrict__ r,
                                                              double* __restrict__ part) {
    double v[2] = {0.0, 0.0};
    CSR_LOOP(i, A.n) {
        const double bi = b[i];
        const double ri = bi - csr_row_dot<double>(A, i, [&](int j) { return x[j]; });
        r[i] = ri;
        v[0] += bi * bi;
        v[1] += ri * ri;
    }
    block_sum_store<2>(v, part, gridDim.x, blockIdx.x);
}

// True-residual refresh r = b - A x in FP64 (mixed form, when requested).
static __global__ void __launch_bounds__(kBlock) k_csr_refresh(const Ctl* __restrict__ ctl, CsrOp<double> A,
                                                        const double* __restrict__ b, const double* __restrict__ x,
                                                        double* __restrict__ r, double* __restrict__ part) {
    if (ctl->state == 2 || !ctl->refresh_req) return;
    double v[1] = {0.0};
    CSR_LOOP(i, A.n) {
        const double ri = b[i] - csr_row_dot<double>(A, i, [&](int j) { return x[j]; });
        r[i] = ri;
        v[0] += ri * ri;
    }
    block_sum_store<1>(v, part, gridDim.x, blockIdx.x);
}

// y = A x (FP64).
static __global__ void __launch_bounds__(kBlock) k_csr_apply(CsrOp<double> A, const double* __restrict__ x,
                                                      double* __restrict__ y) {
    CSR_LOOP(i, A.n) y[i] = csr_row_dot<double>(A, i, [&](int j) { return x[j]; });
}

// Damped Jacobi on a level from c0 = 0 (eq. (2)): c1 = omega g / D; with
// two sweeps c = c1 + omega (g - A c1) / D, c1 formed on the fly.  Output
// to out[i * stride] (a vector, or one column of a node-major block).
template <typename T, typename G>
__device__ __forceinline__ T csr_smooth_at(const CsrOp<T>& A, const T* __restrict__ D, const G* __restrict__ g, int i,
                                           T omega, int two) {
    const T gi = T(g[i]);
    const T c1 = omega * (gi / D[i]);
    T c = c1;
    if (two) {
        const T Ac = csr_row_dot<T>(A, i, [&](int j) { return omega * (T(g[j]) / D[j]); });
        c = c1 + omega * ((gi - Ac) / D[i]);
    }
    return c;
}

template <typename T, typename G>
__global__ void __launch_bounds__(kBlock) k_csr_smooth(const Ctl* __restrict__ ctl, CsrOp<T> A,
                                                       const T* __restrict__ D, const G* __restrict__ g,
                                                       T* __restrict__ out, int stride, T omega, int two) {
    if (ctl->state != 0) return;
    CSR_LOOP(i, A.n) out[(size_t)i * stride] = csr_smooth_at<T, G>(A, D, g, i, omega, two);
}

// One further sweep cout = cin + omega (g - A cin) / D.
template <typename T, typename G>
__global__ void __launch_bounds__(kBlock) k_csr_sweep(const Ctl* __restrict__ ctl, CsrOp<T> A,
                                                      const T* __restrict__ D, const G* __restrict__ g,
                                                      const T* __restrict__ cin, int sin, T* __restrict__ cout,
                                                      int sout, T omega) {
    if (ctl->state != 0) return;
    CSR_LOOP(i, A.n) {
        const T Ac = csr_row_dot<T>(A, i, [&](int j) { return cin[(size_t)j * sin]; });
        cout[(size_t)i * sout] = cin[(size_t)i * sin] + omega * ((T(g[i]) - Ac) / D[i]);
    }
}

// Restriction g = R gf (R = s P^T in CSR, rows = coarse unknowns).
template <typename T, typename TI>
__global__ void __launch_bounds__(kBlock) k_csr_restrict(const Ctl* __restrict__ ctl, CsrOp<T> R,
                                                         const TI* __restrict__ gf, T* __restrict__ g) {
    if (ctl->state != 0) return;
    CSR_LOOP(i, R.n) g[i] = csr_row_dot<T>(R, i, [&](int j) { return T(gf[j]); });
}

// One restriction in blocks [0, nr) (grid-stride over them) and, in the
// blocks after them, the first min(nu, 2) sweeps on a level whose input is
// already in place (the finest level beside the first restriction, both
// reading r; a restricted level beside the restriction from it; nr = 0:
// the smoother alone).  The halves read and write disjoint data.
template <typename T, typename TI, typename G>
__global__ void __launch_bounds__(kBlock) k_csr_restrict_smooth(const Ctl* __restrict__ ctl, CsrOp<T> R,
                                                                const TI* __restrict__ gf, T* __restrict__ gc,
                                                                int nr, CsrOp<T> A, const T* __restrict__ D,
                                                                const G* __restrict__ g, T* __restrict__ out,
                                                                int stride, T omega, int two) {
    if (ctl->state != 0) return;
    const int b = (int)blockIdx.x;
    if (b < nr) {
        for (int i = b * kBlock + (int)threadIdx.x; i < R.n; i += nr * kBlock)
            gc[i] = csr_row_dot<T>(R, i, [&](int j) { return T(gf[j]); });
        return;
    }
    const int bs = b - nr, gs = (int)gridDim.x - nr;
    for (int i = bs * kBlock + (int)threadIdx.x; i < A.n; i += gs * kBlock)
        out[(size_t)i * stride] = csr_smooth_at<T, G>(A, D, g, i, omega, two);
}

// Sum over the 64 lanes of a wavefront (every lane gets the sum; fixed
// order, so deterministic).
template <typename T>
__device__ __forceinline__ T csr_wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Row i's dot product with one wavefront per row: lane l takes entries l,
// l + 64, .. of the row (all loads of a lane issued together), then the
// lanes' sums are added by the butterfly.  For rows of the small coarse
// levels, where one thread per row walks its ~27 entries in dependent
// groups while few rows keep the chip busy.
template <typename T, typename F>
__device__ __forceinline__ T csr_row_dot_wave(const CsrOp<T>& A, int i, F&& u) {
    const int s = i >> 6;
    const int off = A.soff[s] + (i & 63), w = A.swid[s];
    T acc = T(0);
    for (int k = (int)threadIdx.x & 63; k < w; k += 64) acc += A.val[off + 64 * k] * u(A.col[off + 64 * k]);
    return csr_wave_sum(acc);
}

// k_csr_restrict_smooth with the rows of either half taken one per
// wavefront (WR: the restriction's, WS: the smoother's), the same
// arithmetic up to the order of each row's sum.
template <typename T, typename TI, typename G, int WR, int WS>
__global__ void __launch_bounds__(kBlock) k_csr_restrict_smooth_w(const Ctl* __restrict__ ctl, CsrOp<T> R,
                                                                  const TI* __restrict__ gf, T* __restrict__ gc,
                                                                  int nr, CsrOp<T> A, const T* __restrict__ D,
                                                                  const G* __restrict__ g, T* __restrict__ out,
                                                                  int stride, T omega, int two) {
    if (ctl->state != 0) return;
    const int b = (int)blockIdx.x, wv = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
    if (b < nr) {
        if (WR) {
            for (int i = b * kWaves + wv; i < R.n; i += nr * kWaves) {
                const T v = csr_row_dot_wave<T>(R, i, [&](int j) { return T(gf[j]); });
                if (lane == 0) gc[i] = v;
            }
        } else {
            for (int i = b * kBlock + (int)threadIdx.x; i < R.n; i += nr * kBlock)
                gc[i] = csr_row_dot<T>(R, i, [&](int j) { return T(gf[j]); });
        }
        return;
    }
    const int bs = b - nr, gs = (int)gridDim.x - nr;
    if (WS) {
        for (int i = bs * kWaves + wv; i < A.n; i += gs * kWaves) {
            const T gi = T(g[i]), Di = D[i];
            const T c1 = omega * (gi / Di);
            T c = c1;
            if (two) {
                const T Ac = csr_row_dot_wave<T>(A, i, [&](int j) { return omega * (T(g[j]) / D[j]); });
                c = c1 + omega * ((gi - Ac) / Di);
            }
            if (lane == 0) out[(size_t)i * stride] = c;
        }
    } else {
        for (int i = bs * kBlock + (int)threadIdx.x; i < A.n; i += gs * kBlock)
            out[(size_t)i * stride] = csr_smooth_at<T, G>(A, D, g, i, omega, two);
    }
}

// Block carry up one level: Yf[:, 0..NC-1] = P Yc[:, 0..NC-1] (node-major,
// strides even_up(NC) and even_up(NC+1)).
template <typename T, int NC>
__global__ void __launch_bounds__(kBlock) k_csr_prolong(const Ctl* __restrict__ ctl, CsrOp<T> P,
                                                        const T* __restrict__ Yc, T* __restrict__ Yf) {
    if (ctl->state != 0) return;
    constexpr int SC = even_up(NC), SF = even_up(NC + 1);
    CSR_LOOP(i, P.n) {
        T acc[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] = T(0);
        for_row(P, i, [&](int j, T w) {
            const T* y = Yc + (size_t)j * SC;
#pragma unroll
            for (int c = 0; c < NC; ++c) acc[c] += w * y[c];
        });
#pragma unroll
        for (int c = 0; c < NC; ++c) Yf[(size_t)i * SF + c] = acc[c];
    }
}

// The NB level corrections at fine row i: z[c] = (P_{L-1} Y_{L-1})_{i,c} for
// c < NB-1, z[NB-1] = cL[i].
template <typename T, int NB>
__device__ __forceinline__ void csr_fine_z(const CsrOp<T>& P, const T* __restrict__ Y, const T* __restrict__ cL,
                                           int i, T (&z)[NB]) {
    if constexpr (NB > 1) {
        constexpr int SY = even_up(NB - 1);
#pragma unroll
        for (int c = 0; c < NB - 1; ++c) z[c] = T(0);
        for_row(P, i, [&](int j, T w) {
            const T* y = Y + (size_t)j * SY;
#pragma unroll
            for (int c = 0; c < NB - 1; ++c) z[c] += w * y[c];
        });
    }
    z[NB - 1] = cL[i];
}

// W = Q^T Z partial sums (NB x NB).
template <typename T, int NB>
__global__ void __launch_bounds__(kBlock) k_csr_fine_W(const Ctl* __restrict__ ctl, int N, CsrOp<T> P,
                                                       const T* __restrict__ Y, const T* __restrict__ cL,
                                                       const T* __restrict__ Q, double* __restrict__ part) {
    if (ctl->state != 0) return;
    constexpr int S = even_up(NB);
    double w[NB * NB];
#pragma unroll
    for (int q = 0; q < NB * NB; ++q) w[q] = 0.0;
    CSR_LOOP(i, N) {
        T z[NB];
        csr_fine_z<T, NB>(P, Y, cL, i, z);
        T q[S];
        load_node<T, S>(Q + (size_t)i * S, q);
#pragma unroll
        for (int a = 0; a < NB; ++a) {
            const double qa = double(q[a]);
#pragma unroll
            for (int c = 0; c < NB; ++c) w[a * NB + c] += qa * double(z[c]);
        }
    }
    block_sum_store<NB * NB>(w, part, gridDim.x, blockIdx.x);
}

// x += P_k alpha_k; unless stopping, P_{k+1} = Z - sum_j P_j beta_j over the
// m stored blocks (slot cur holds P_k), into slot nxt; init: P_0 = Z_0.
template <typename T, int NB>
__global__ void __launch_bounds__(kBlock) k_csr_update_xP(const Ctl* __restrict__ ctl, int N, CsrOp<T> P,
                                                          const T* __restrict__ Y, const T* __restrict__ cL,
                                                          PWin<T> win, int m, int cur, int nxt,
                                                          double* __restrict__ x, const double* __restrict__ alpha,
                                                          const double* __restrict__ beta, int init) {
    const int state = ctl->state;
    if (state == 2 || (init && state != 0)) return;
    constexpr int S = even_up(NB);
    __shared__ double sab[NB + kMaxWin * NB * NB];
    if (!init) {
        for (int q = threadIdx.x; q < NB + m * NB * NB; q += kBlock) {
            if (q < NB) {
                sab[q] = alpha[q];
            } else {
                const int j = (q - NB) / (NB * NB), e = (q - NB) - j * NB * NB;
                sab[q] = beta[(size_t)j * kMaxNB * kMaxNB + e];
            }
        }
    }
    __syncthreads();
    T* __restrict__ Pc = win.p[cur];
    T* __restrict__ Pn = win.p[nxt];
    CSR_LOOP(i, N) {
        T pk[S];
        if (!init) {
            load_node<T, S>(Pc + (size_t)i * S, pk);
            double xi = x[i];
#pragma unroll
            for (int c = 0; c < NB; ++c) xi += double(pk[c]) * sab[c];
            x[i] = xi;
            if (state != 0) continue;
        }
        T z[NB];
        csr_fine_z<T, NB>(P, Y, cL, i, z);
        double v[NB];
#pragma unroll
        for (int c = 0; c < NB; ++c) v[c] = double(z[c]);
        if (!init) {
            const double* bc = sab + NB + cur * NB * NB;
#pragma unroll
            for (int c = 0; c < NB; ++c)
#pragma unroll
                for (int a2 = 0; a2 < NB; ++a2) v[c] -= double(pk[a2]) * bc[a2 * NB + c];
            for (int j = 0; j < m; ++j) {
                if (j == cur) continue;
                T pj[S];
                load_node<T, S>(win.p[j] + (size_t)i * S, pj);
                const double* bj = sab + NB + j * NB * NB;
#pragma unroll
                for (int c = 0; c < NB; ++c)
#pragma unroll
                    for (int a2 = 0; a2 < NB; ++a2) v[c] -= double(pj[a2]) * bj[a2 * NB + c];
            }
        }
        T pn[S];
#pragma unroll
        for (int c = 0; c < NB; ++c) pn[c] = T(v[c]);
#pragma unroll
        for (int c = NB; c < S; ++c) pn[c] = T(0);
        store_node<T, S>(Pn + (size_t)i * S, pn);
    }
}

// Q = A P, partial Gram upper triangle and P^T r.
template <typename T, int NB>
__global__ void __launch_bounds__(kBlock) k_csr_spmm_gram(const Ctl* __restrict__ ctl, CsrOp<T> A,
                                                          const T* __restrict__ P, T* __restrict__ Q,
                                                          const double* __restrict__ r, double* __restrict__ part) {
    if (ctl->state != 0) return;
    constexpr int NG = NB * (NB + 1) / 2;
    constexpr int S = even_up(NB);
    double acc[NG + NB];
#pragma unroll
    for (int q = 0; q < NG + NB; ++q) acc[q] = 0.0;
    CSR_LOOP(i, A.n) {
        T q[S], pv[S], nb[S];
#pragma unroll
        for (int c = 0; c < S; ++c) q[c] = T(0);
        for_row(A, i, [&](int j, T w) {
            load_node<T, S>(P + (size_t)j * S, nb);
#pragma unroll
            for (int c = 0; c < S; ++c) q[c] += w * nb[c];
        });
        store_node<T, S>(Q + (size_t)i * S, q);
        load_node<T, S>(P + (size_t)i * S, pv);
        const double ri = r[i];
        int g = 0;
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int c = a; c < NB; ++c) acc[g++] += double(pv[a]) * double(q[c]);
#pragma unroll
        for (int a = 0; a < NB; ++a) acc[NG + a] += double(pv[a]) * ri;
    }
    block_sum_store<NG + NB>(acc, part, gridDim.x, blockIdx.x);
}

// Explicit Z (widened to double, column-major), for the mg_block entry point.
template <typename T, int NB>
__global__ void __launch_bounds__(kBlock) k_csr_write_Z(int N, CsrOp<T> P, const T* __restrict__ Y,
                                                        const T* __restrict__ cL, double* __restrict__ Z) {
    CSR_LOOP(i, N) {
        T z[NB];
        csr_fine_z<T, NB>(P, Y, cL, i, z);
#pragma unroll
        for (int c = 0; c < NB; ++c) Z[(size_t)c * N + i] = double(z[c]);
    }
}

#undef CSR_LOOP

}  // namespace amg
