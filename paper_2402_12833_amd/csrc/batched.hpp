// Batched MPCG: many independent structured Poisson problems (each with its
// own grid size, hierarchy and right-hand side) solved together.  Every
// step of Algorithm 1 is one launch over all problems of a group (the
// problems with the same number of levels, so that the number of directions
// is a compile-time constant): each block belongs to one problem, found
// through a block map built on the host, and works on a contiguous node
// range of one level of it.  Each problem has its own control word, step
// coefficients and partial sums (value-major rows of its own block count),
// so the single-block reductions of the one-problem solver run unchanged,
// one block per problem.  Problems that have stopped skip every launch.
// The launches of k_poll iterations of all groups are captured in one HIP
// graph; the host polls the control words between graph launches.
#pragma once

#include "common.hpp"
#include "grid_kernels.hpp"
#include "small_kernels.hpp"

namespace amg {

constexpr int kBChunk = 4 * kBlock;   // fine nodes per block of the batched fine kernels

// Partial-sum rows of one problem (in units of its block count pcnt).
constexpr int kBPartInit = 0;                              // ||b||^2, ||r||^2
constexpr int kBPartRho = 2;                               // ||r||^2
constexpr int kBPartW = 3;                                 // W, kMaxNB^2 rows
constexpr int kBPartG = 3 + kMaxNB * kMaxNB;               // Gram + P^T r
constexpr int kBPartRef = kBPartG + kMaxNB * (kMaxNB + 1) / 2 + kMaxNB;   // refresh ||r||^2
constexpr int kBPartRows = kBPartRef + 1;

// Step coefficients of one problem: alpha, beta, G^+.
constexpr int kBSmall = kMaxNB + 2 * kMaxNB * kMaxNB;

template <typename T>
struct BInst {
    int nlev;
    int n[kMaxLevels], N[kMaxLevels];   // per level, coarsest first
    FineOp<T> op;                       // finest operator (constant coefficient)
    FineOp<double> op64;                // the same in FP64 (residual, refresh)
    double *x, *r, *b;
    T *P, *Q, *cL;                      // node-major blocks (stride even_up(nlev)), finest smoother output
    const T* coef[kMaxLevels];          // coarse operators, coefficient-major
    T* g[kMaxLevels];                   // restricted residuals
    T* c1[kMaxLevels];                  // first smoothing sweep omega g / D
    T* Y[kMaxLevels];                   // block carry [P Y_{l-1} | c_l]
    Ctl* ctl;
    double* small;                      // alpha, beta, G^+ (kBSmall)
    double* part;                       // kBPartRows rows of pcnt partial sums
    int pcnt;                           // blocks of this problem in the fine launches
};

// A block's problem (index into the instance array), its block index within
// that problem (fine launches) and its node range.
struct BBlk {
    int inst, blk, start, end;
};

template <typename T>
__device__ __forceinline__ double* bpart(const BInst<T>& I, int row) {
    return I.part + (size_t)row * I.pcnt;
}

// ---------------------------------------------------------- fine level

// r = b - A x (FP64), partial ||b||^2 and ||r||^2.
template <int DIM, typename T>
__global__ void __launch_bounds__(kBlock) k_b_init_residual(const BInst<T>* __restrict__ insts,
                                                            const BBlk* __restrict__ map) {
    const BBlk m = map[blockIdx.x];
    const BInst<T>& I = insts[m.inst];
    const int n = I.n[I.nlev - 1];
    double v[2] = {0.0, 0.0};
    for (int idx = m.start + threadIdx.x; idx < m.end; idx += kBlock) {
        const Idx<DIM> p = decomp<DIM>(idx, n);
        const double bi = I.b[idx];
        const double ri = bi - fine_apply<DIM, double>(I.op64, I.x, idx, p);
        I.r[idx] = ri;
        v[0] += bi * bi;
        v[1] += ri * ri;
    }
    block_sum_store<2>(v, bpart(I, kBPartInit), I.pcnt, m.blk);
}

// b == 0: x = 0.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_b_zero_if(const BInst<T>* __restrict__ insts,
                                                      const BBlk* __restrict__ map) {
    const BBlk m = map[blockIdx.x];
    const BInst<T>& I = insts[m.inst];
    if (!I.ctl->zero_x) return;
    for (int idx = m.start + threadIdx.x; idx < m.end; idx += kBlock) I.x[idx] = 0.0;
}

// r -= Q alpha, partial ||r||^2.
template <typename T, int NB>
__global__ void __launch_bounds__(kBlock) k_b_update_r(const BInst<T>* __restrict__ insts,
                                                       const BBlk* __restrict__ map) {
    const BBlk m = map[blockIdx.x];
    const BInst<T>& I = insts[m.inst];
    if (I.ctl->state != 0) return;
    constexpr int S = even_up(NB);
    double a[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) a[c] = I.small[c];
    double v[1] = {0.0};
    for (int idx = m.start + threadIdx.x; idx < m.end; idx += kBlock) {
        T q[S];
        load_node<T, S>(I.Q + (size_t)idx * S, q);
        double ri = I.r[idx];
#pragma unroll
        for (int c = 0; c < NB; ++c) ri -= double(q[c]) * a[c];
        I.r[idx] = ri;
        v[0] += ri * ri;
    }
    block_sum_store<1>(v, bpart(I, kBPartRho), I.pcnt, m.blk);
}

// Finest smoother output cL = S^nu r (nu = 1 or 2 sweeps from zero).
template <int DIM, typename T>
__device__ __forceinline__ void b_fine_smooth_block(const BInst<T>* __restrict__ insts, const BBlk& m, T omega,
                                                    int two) {
    const BInst<T>& I = insts[m.inst];
    if (I.ctl->state != 0) return;
    const int n = I.n[I.nlev - 1];
    for (int idx = m.start + threadIdx.x; idx < m.end; idx += kBlock) {
        const Idx<DIM> p = decomp<DIM>(idx, n);
        I.cL[idx] = fine_smooth_at<DIM, T, double>(I.op, I.r, idx, p, omega, two);
    }
}

template <int DIM, typename T>
__global__ void __launch_bounds__(kBlock) k_b_fine_smooth(const BInst<T>* __restrict__ insts,
                                                          const BBlk* __restrict__ map, T omega, int two) {
    b_fine_smooth_block<DIM, T>(insts, map[blockIdx.x], omega, two);
}

// W = Q^T Z partial sums (NB x NB), Z from the level-(L-1) block carry and cL.
template <int DIM, typename T, int NB>
__global__ void __launch_bounds__(kBlock) k_b_fine_W(const BInst<T>* __restrict__ insts,
                                                     const BBlk* __restrict__ map) {
    const BBlk m = map[blockIdx.x];
    const BInst<T>& I = insts[m.inst];
    if (I.ctl->state != 0) return;
    constexpr int S = even_up(NB);
    const int L = I.nlev - 1, n = I.n[L];
    const T* Yc = L > 0 ? I.Y[L - 1] : nullptr;
    const int nc = L > 0 ? I.n[L - 1] : 1;
    double w[NB * NB];
#pragma unroll
    for (int q = 0; q < NB * NB; ++q) w[q] = 0.0;
    for (int idx = m.start + threadIdx.x; idx < m.end; idx += kBlock) {
        const Idx<DIM> p = decomp<DIM>(idx, n);
        T z[NB];
        fine_z<DIM, T, NB, 0>(Yc, nc, I.cL, nullptr, false, idx, p, z);
        T q[S];
        load_node<T, S>(I.Q + (size_t)idx * S, q);
#pragma unroll
        for (int a = 0; a < NB; ++a) {
            const double qa = double(q[a]);
#pragma unroll
            for (int c = 0; c < NB; ++c) w[a * NB + c] += qa * double(z[c]);
        }
    }
    block_sum_store<NB * NB>(w, bpart(I, kBPartW), I.pcnt, m.blk);
}

// x += P alpha (deferred); then, unless stopping, P = Z - P beta in place.
// init = 1: P_0 = Z_0 only.
template <int DIM, typename T, int NB>
__global__ void __launch_bounds__(kBlock) k_b_update_xP(const BInst<T>* __restrict__ insts,
                                                        const BBlk* __restrict__ map, int init) {
    const BBlk m = map[blockIdx.x];
    const BInst<T>& I = insts[m.inst];
    const int state = I.ctl->state;
    if (state == 2 || (init && state != 0)) return;
    constexpr int S = even_up(NB);
    const int L = I.nlev - 1, n = I.n[L];
    const T* Yc = L > 0 ? I.Y[L - 1] : nullptr;
    const int nc = L > 0 ? I.n[L - 1] : 1;
    __shared__ double sab[NB + NB * NB];
    if (!init) {
        for (int q = threadIdx.x; q < NB + NB * NB; q += kBlock)
            sab[q] = q < NB ? I.small[q] : I.small[kMaxNB + q - NB];
    }
    __syncthreads();
    for (int idx = m.start + threadIdx.x; idx < m.end; idx += kBlock) {
        T pk[S];
        if (!init) {
            load_node<T, S>(I.P + (size_t)idx * S, pk);
            double xi = I.x[idx];
#pragma unroll
            for (int c = 0; c < NB; ++c) xi += double(pk[c]) * sab[c];
            I.x[idx] = xi;
            if (state != 0) continue;
        }
        const Idx<DIM> p = decomp<DIM>(idx, n);
        T z[NB];
        fine_z<DIM, T, NB, 0>(Yc, nc, I.cL, nullptr, false, idx, p, z);
        T pn[S];
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            double v = double(z[c]);
            if (!init) {
#pragma unroll
                for (int a2 = 0; a2 < NB; ++a2) v -= double(pk[a2]) * sab[NB + a2 * NB + c];
            }
            pn[c] = T(v);
        }
#pragma unroll
        for (int c = NB; c < S; ++c) pn[c] = T(0);
        store_node<T, S>(I.P + (size_t)idx * S, pn);
    }
}

// True-residual refresh r = b - A x in FP64 (mixed form, when requested).
template <int DIM, typename T>
__global__ void __launch_bounds__(kBlock) k_b_refresh(const BInst<T>* __restrict__ insts,
                                                      const BBlk* __restrict__ map) {
    const BBlk m = map[blockIdx.x];
    const BInst<T>& I = insts[m.inst];
    if (I.ctl->state == 2 || !I.ctl->refresh_req) return;
    const int n = I.n[I.nlev - 1];
    double v[1] = {0.0};
    for (int idx = m.start + threadIdx.x; idx < m.end; idx += kBlock) {
        const Idx<DIM> p = decomp<DIM>(idx, n);
        const double ri = I.b[idx] - fine_apply<DIM, double>(I.op64, I.x, idx, p);
        I.r[idx] = ri;
        v[0] += ri * ri;
    }
    block_sum_store<1>(v, bpart(I, kBPartRef), I.pcnt, m.blk);
}

// Q = A P, partial Gram upper triangle and P^T r.
template <int DIM, typename T, int NB>
__global__ void __launch_bounds__(kBlock) k_b_spmm_gram(const BInst<T>* __restrict__ insts,
                                                        const BBlk* __restrict__ map) {
    const BBlk m = map[blockIdx.x];
    const BInst<T>& I = insts[m.inst];
    if (I.ctl->state != 0) return;
    constexpr int NG = NB * (NB + 1) / 2;
    constexpr int S = even_up(NB);
    const int n = I.n[I.nlev - 1];
    double acc[NG + NB];
#pragma unroll
    for (int q = 0; q < NG + NB; ++q) acc[q] = 0.0;
    for (int idx = m.start + threadIdx.x; idx < m.end; idx += kBlock) {
        const Idx<DIM> p = decomp<DIM>(idx, n);
        T pv[S], qv[S];
        fine_apply_block<DIM, T, S>(I.op, I.P, idx, p, pv, qv);
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
    block_sum_store<NG + NB>(acc, bpart(I, kBPartG), I.pcnt, m.blk);
}

// ---------------------------------------------------------- coarse levels

// Restriction to level l (thread per coarse node) and the first sweep
// c1 = omega g / D; FINE: from the finest residual r.
template <int DIM, typename T, bool FINE>
__device__ __forceinline__ void b_restrict_block(const BInst<T>* __restrict__ insts, const BBlk& m, int l, T omega) {
    const BInst<T>& I = insts[m.inst];
    if (I.ctl->state != 0) return;
    const int idx = m.start + threadIdx.x;
    if (idx >= m.end) return;
    T g;
    if constexpr (FINE) g = restrict_at<DIM, double, T>(I.r, I.n[l + 1], I.n[l], idx);
    else g = restrict_at<DIM, T, T>(I.g[l + 1], I.n[l + 1], I.n[l], idx);
    const T* D = I.coef[l] + (size_t)stencil_center<DIM>() * I.N[l];
    I.g[l][idx] = g;
    I.c1[l][idx] = omega * (g / D[idx]);
}

// Damped Jacobi on level l (nu = 1 or 2 sweeps from zero) into the last
// column of the level's block carry.
template <int DIM, typename T>
__device__ __forceinline__ void b_coarse_smooth_block(const BInst<T>* __restrict__ insts, const BBlk& m, int l,
                                                      T omega, int two) {
    const BInst<T>& I = insts[m.inst];
    if (I.ctl->state != 0) return;
    const int idx = m.start + threadIdx.x;
    if (idx >= m.end) return;
    CoarseOp<T> op{I.n[l], I.N[l], I.coef[l], 0};
    I.Y[l][(size_t)idx * even_up(l + 1) + l] =
        coarse_smooth_at<DIM, T>(op, I.g[l], I.c1[l], nullptr, idx, omega, 0, two);
}

// The chain of every group in the same launches: a coarse level is named by
// its depth below the finest one (level l = nlev - 1 - depth of each
// problem), so one launch serves the problems of all level counts.  As for
// a single problem the smoothers run inside the restriction launches:
// blocks [0, nr) restrict into depth dr with map mr (depth 1: from r), the
// blocks after them smooth with map ms, the finest level
// (k_b_dep_restrict_fine_smooth) or depth ds, which the previous launch
// restricted into (k_b_dep_restrict_coarse_smooth; nr = 0: smoothing only).
// The two halves read and write disjoint data.
template <typename T>
__device__ __forceinline__ int b_level(const BInst<T>* __restrict__ insts, const BBlk& m, int depth) {
    return insts[m.inst].nlev - 1 - depth;
}

template <int DIM, typename T>
__global__ void __launch_bounds__(kBlock) k_b_dep_restrict_fine_smooth(const BInst<T>* __restrict__ insts,
                                                                       const BBlk* __restrict__ mr, int nr,
                                                                       const BBlk* __restrict__ ms, T omega,
                                                                       int two) {
    if ((int)blockIdx.x < nr) {
        const BBlk m = mr[blockIdx.x];
        b_restrict_block<DIM, T, true>(insts, m, b_level(insts, m, 1), omega);
    } else {
        b_fine_smooth_block<DIM, T>(insts, ms[blockIdx.x - nr], omega, two);
    }
}

template <int DIM, typename T>
__global__ void __launch_bounds__(kBlock) k_b_dep_restrict_coarse_smooth(const BInst<T>* __restrict__ insts,
                                                                         const BBlk* __restrict__ mr, int nr,
                                                                         int dr, const BBlk* __restrict__ ms,
                                                                         int ds, T omega, int two) {
    if ((int)blockIdx.x < nr) {
        const BBlk m = mr[blockIdx.x];
        b_restrict_block<DIM, T, false>(insts, m, b_level(insts, m, dr), omega);
    } else {
        const BBlk m = ms[blockIdx.x - nr];
        b_coarse_smooth_block<DIM, T>(insts, m, b_level(insts, m, ds), omega, two);
    }
}

// Block carry into depth d from depth d + 1: Y_{l+1}[:, 0..l] = P Y_l with
// l + 1 = nlev - 1 - d, the column count chosen per problem.
template <int DIM, typename T>
__global__ void __launch_bounds__(kBlock) k_b_dep_prolong(const BInst<T>* __restrict__ insts,
                                                          const BBlk* __restrict__ map, int d) {
    const BBlk m = map[blockIdx.x];
    const BInst<T>& I = insts[m.inst];
    if (I.ctl->state != 0) return;
    const int idx = m.start + threadIdx.x;
    if (idx >= m.end) return;
    const int l = I.nlev - 2 - d;
    switch (l + 1) {
        case 1: prolong_at<DIM, T, 1>(I.Y[l], I.n[l], I.Y[l + 1], I.n[l + 1], idx); break;
        case 2: prolong_at<DIM, T, 2>(I.Y[l], I.n[l], I.Y[l + 1], I.n[l + 1], idx); break;
        case 3: prolong_at<DIM, T, 3>(I.Y[l], I.n[l], I.Y[l + 1], I.n[l + 1], idx); break;
        case 4: prolong_at<DIM, T, 4>(I.Y[l], I.n[l], I.Y[l + 1], I.n[l + 1], idx); break;
        case 5: prolong_at<DIM, T, 5>(I.Y[l], I.n[l], I.Y[l + 1], I.n[l + 1], idx); break;
        case 6: prolong_at<DIM, T, 6>(I.Y[l], I.n[l], I.Y[l + 1], I.n[l + 1], idx); break;
        default: prolong_at<DIM, T, 7>(I.Y[l], I.n[l], I.Y[l + 1], I.n[l + 1], idx); break;
    }
}

// ---------------------------------------------------------- reductions
// One block per problem (block b works on instance first + b): the
// one-problem reduction logic on that problem's partial rows.

template <typename T>
__global__ void __launch_bounds__(kRedBlock) k_b_reduce_init(const BInst<T>* __restrict__ insts, double tol) {
    const BInst<T>& I = insts[blockIdx.x];
    reduce_init_body(I.ctl, bpart(I, kBPartInit), I.pcnt, tol, nullptr);
}

template <typename T, int NB>
__global__ void __launch_bounds__(kRedBlock) k_b_reduce_beta(const BInst<T>* __restrict__ insts, int first,
                                                          int mixed) {
    const BInst<T>& I = insts[first + blockIdx.x];
    reduce_beta_body<NB>(I.ctl, bpart(I, kBPartRho), I.pcnt, bpart(I, kBPartW), I.pcnt, 1, 0,
                         I.small + kMaxNB + kMaxNB * kMaxNB, I.small + kMaxNB, nullptr, mixed);
}

template <typename T, int NB>
__global__ void __launch_bounds__(kRedBlock) k_b_reduce_alpha(const BInst<T>* __restrict__ insts, int first) {
    const BInst<T>& I = insts[first + blockIdx.x];
    reduce_alpha_body<NB>(I.ctl, bpart(I, kBPartG), I.pcnt, I.small + kMaxNB + kMaxNB * kMaxNB, I.small, nullptr);
}

template <typename T>
__global__ void __launch_bounds__(kRedBlock) k_b_refresh_reduce(const BInst<T>* __restrict__ insts, int first) {
    const BInst<T>& I = insts[first + blockIdx.x];
    refresh_reduce_body(I.ctl, bpart(I, kBPartRef), I.pcnt, nullptr);
}

}  // namespace amg
