// Shared device helpers: control word, launch geometry, deterministic
// block reductions.  gfx950: 64-wide wavefronts, 256-thread blocks.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace amg {

constexpr int kBlock = 256;        // threads per block (4 wavefronts)
constexpr int kWaves = kBlock / 64;
constexpr int kMaxLevels = 8;
constexpr int kMaxNB = 8;          // search directions per iteration (L + 1 [+ 1])
constexpr int kMaxWin = 8;         // truncation window m: direction blocks kept
constexpr int kNumXcd = 8;         // MI355X: 8 XCDs, blocks dispatched round-robin

// Solver control word in device memory.  Only single-block kernels write it;
// every other kernel reads `state` once at entry and exits early unless the
// iteration is still running, so iterations launched after convergence are
// no-ops and the count stays exact.
struct Ctl {
    int state;        // 0 running, 1 stop after the pending x update, 2 finished
    int it;           // number of x updates
    int status;       // AMGMPCG_* status once finished
    int refreshes;    // true-residual refreshes (FP32 bulk)
    int refresh_req;  // 1: refresh r = b - A x after this iteration's x update
    int rank;         // rank of the last Gram pseudo-inverse
    int maxit;
    int zero_x;       // 1: b == 0, the solution is x = 0
    int hist_cap;     // capacity of the history buffers (iterations)
    int pad0, pad1, pad2;
    double bnorm2;    // ||b||^2
    double tol2;      // tol^2 ||b||^2
    double rho;       // ||r||^2 of the current residual
    double rho_ref;   // ||r||^2 at the last refresh
    double drop2;     // refresh_drop^2
    double tau;       // eigenvalue cut of the unit-diagonal Gram
    double relres_true;   // ||b - A x||_2 / ||b||_2 of the returned x (FP64), when computed
    double tol;           // relative tolerance (read by the persistent batched launch)
};

// Logical block index so that each XCD (blockIdx % 8) owns a contiguous range
// of logical blocks, hence a contiguous slab of the grid: stencil neighbours in
// y and z are then mostly produced and consumed inside the same XCD's L2.
__device__ __forceinline__ int xcd_block_of(int b, int nblocks) {
    if (nblocks % kNumXcd) return b;
    return (b % kNumXcd) * (nblocks / kNumXcd) + b / kNumXcd;
}

__device__ __forceinline__ int xcd_block(int nblocks) { return xcd_block_of((int)blockIdx.x, nblocks); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Smallest power of two >= k (k <= 64).
__host__ __device__ constexpr int pow2_up(int k) { return k <= 1 ? 1 : 2 * pow2_up((k + 1) / 2); }

// Reduce K values per lane over the 64 lanes of a wavefront by recursive
// halving: at distance d = 32, 16, ... each lane keeps one half of its value
// list and adds the partner's copy of that half, so K values cost about K
// shuffles instead of 6 K.  Afterwards lane l holds the wave sum of value
// index vidx(l) in v[0] (lanes sharing an index hold the same sum).  The
// order of additions is fixed, so the result is deterministic.
template <int K>
__device__ __forceinline__ int wave_reduce_multi(double (&v)[K]) {
    constexpr int KP = pow2_up(K);
    constexpr int LOG = KP == 1 ? 0 : KP == 2 ? 1 : KP == 4 ? 2 : KP == 8 ? 3 : KP == 16 ? 4 : KP == 32 ? 5 : 6;
    const int lane = threadIdx.x & 63;
    int vidx = 0;
#pragma unroll
    for (int s = 0; s < LOG; ++s) {
        const int half = KP >> (s + 1), d = 32 >> s;
        const bool up = (lane & d) != 0;
#pragma unroll
        for (int i = 0; i < KP / 2; ++i) {
            if (i < half && i < K) {
                // values past K (padding of the first step) are zero
                const double lo = v[i];
                const double hi = (i + half < K) ? v[(i + half < K) ? i + half : 0] : 0.0;
                const double send = up ? lo : hi;
                const double keep = up ? hi : lo;
                v[i] = keep + __shfl_xor(send, d);
            }
        }
        vidx = 2 * vidx + (up ? 1 : 0);
    }
    // remaining distances: plain butterfly on the single value
#pragma unroll
    for (int s = LOG; s < 6; ++s) v[0] += __shfl_xor(v[0], 32 >> s);
    return vidx;
}

// Sum K per-thread values over the block in a fixed order and store value k
// of logical block lb at part[k * nblk + lb] (value-major, so that the final
// reduction reads each value's partials contiguously).
template <int K>
__device__ __forceinline__ void block_sum_store(const double (&v)[K], double* part, int nblk, int lb) {
    constexpr int KP = pow2_up(K);
    __shared__ double sh[kWaves][KP];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double t[K];
#pragma unroll
    for (int k = 0; k < K; ++k) t[k] = v[k];
    const int vi = wave_reduce_multi<K>(t);
    // lanes holding the same index carry the same sum; the lowest one writes
    if ((lane & (64 / KP - 1)) == 0) sh[w][vi] = t[0];
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += kBlock) {
        double s = sh[0][k];
#pragma unroll
        for (int q = 1; q < kWaves; ++q) s += sh[q][k];
        part[(size_t)k * nblk + lb] = s;
    }
    __syncthreads();
}

constexpr int kRedBlock = 1024;    // threads of the single-block reduction kernels
constexpr int kRedWaves = kRedBlock / 64;

// Sum K per-thread values over a block of BS threads into res[0 .. K)
// (shared): the waves reduce by recursive halving, then the wave sums are
// added in wave order.  Fixed order: deterministic.
template <int K, int BS>
__device__ __forceinline__ void block_reduce_bs(double (&v)[K], double* res) {
    constexpr int KP = pow2_up(K);
    constexpr int NW = BS / 64;
    __shared__ double sh[NW][KP];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int vi = wave_reduce_multi<K>(v);
    if ((lane & (64 / KP - 1)) == 0) sh[w][vi] = v[0];
    __syncthreads();
    for (int k = t; k < K; k += BS) {
        double s = sh[0][k];
#pragma unroll
        for (int q = 1; q < NW; ++q) s += sh[q][k];
        res[k] = s;
    }
    __syncthreads();
}

// Thread t's sum of rows t, t + kRedBlock, ... of each of K value-major
// partial arrays part[k * nblk + b] (b < nblk), fixed order.  For
// nblk <= kRedBlock that is one load per value, all issued together.
template <int K>
__device__ __forceinline__ void partial_rows(const double* __restrict__ part, int nblk, double (&v)[K]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = 0.0;
    if (t < nblk) {
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = part[(size_t)k * nblk + t];
    }
    for (int b = t + kRedBlock; b < nblk; b += kRedBlock) {
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] += part[(size_t)k * nblk + b];
    }
}

// Sum K per-thread values over a kRedBlock block into res[0 .. count)
// (shared): the waves reduce by recursive halving, then the wave sums are
// added in wave order.  Fixed order: deterministic.
template <int K>
__device__ __forceinline__ void block_reduce(double (&v)[K], double* res, int count = K) {
    constexpr int KP = pow2_up(K);
    __shared__ double sh[kRedWaves][KP];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int vi = wave_reduce_multi<K>(v);
    if ((lane & (64 / KP - 1)) == 0) sh[w][vi] = v[0];
    __syncthreads();
    for (int k = t; k < count; k += kRedBlock) {
        double s = sh[0][k];
#pragma unroll
        for (int q = 1; q < kRedWaves; ++q) s += sh[q][k];
        res[k] = s;
    }
    __syncthreads();
}

// Reduce the value-major partials part[k * nblk + b] of K values into res[k]
// (shared memory); groups of up to 40 values (values K0 .. K0 + GK - 1 here,
// the rest in the next group), each with its loads in flight together.  Every
// group's size is a compile-time constant, so its per-thread sums stay in
// registers.
template <int K, int K0 = 0>
__device__ __forceinline__ void reduce_partials(const double* __restrict__ part, int nblk,
                                                double* res /* shared, K */) {
    constexpr int GK = K - K0 <= 40 ? K - K0 : 32;
    double v[GK];
    partial_rows<GK>(part + (size_t)K0 * nblk, nblk, v);
    block_reduce<GK>(v, res + K0);
    if constexpr (K0 + GK < K) reduce_partials<K, K0 + GK>(part, nblk, res);
}

}  // namespace amg
