// Structured-grid kernels of one MPCG iteration (Sec. 2, Algorithm 1).
//
// Layout in HBM (all levels): one value per node, flat index i + n*(j + n*k)
// (x fastest); a block of b directions is b such vectors back to back
// (column-major, leading dimension N).  Coarse operators are 3^d-point
// stencils stored coefficient-major: coef[s*N + idx] = A(idx, idx + o_s) with
// s = (dz+1)*9 + (dy+1)*3 + (dx+1).  The finest operator is either the
// constant 2d+1-point Laplacian (only h^-2 stored) or four face arrays
// D, ex, ey, ez with e*[idx] = -A(idx, idx + e_*).
//
// T is the bulk type (double, or float in the mixed form); x, r, b, the Gram
// sums and all reductions are double.  Fine-level kernels are grid-stride
// loops over a fixed grid so that block partial sums have a fixed count and
// the reductions are deterministic.
#pragma once

#include "common.hpp"

namespace amg {

// ------------------------------------------------------------------ indexing

template <int DIM>
struct Idx {
    int i, j, k;
};

template <int DIM>
__device__ __forceinline__ Idx<DIM> decomp(int idx, int n) {
    Idx<DIM> p;
    if (DIM == 2) {
        p.j = idx / n;
        p.i = idx - p.j * n;
        p.k = 0;
    } else {
        int t = idx / n;
        p.i = idx - t * n;
        p.k = t / n;
        p.j = t - p.k * n;
    }
    return p;
}

// ------------------------------------------------------------ fine operator

template <typename T>
struct FineOp {
    int n, N;
    T s0;                  // h^-2 (constant coefficient) — used when D == nullptr
    const T* D;            // variable coefficient: diagonal
    const T* ex;           // coupling to +x neighbour (positive)
    const T* ey;
    const T* ez;
};

template <int DIM, typename T>
__device__ __forceinline__ T fine_diag(const FineOp<T>& op, int idx) {
    return op.D ? op.D[idx] : T(2 * DIM) * op.s0;
}

// (A u)_idx on the finest level, computed in type C.
template <int DIM, typename C, typename T, typename U>
__device__ __forceinline__ C fine_apply(const FineOp<T>& op, const U* __restrict__ u, int idx,
                                        const Idx<DIM>& p) {
    const int n = op.n;
    const int sy = n, sz = n * n;
    if (!op.D) {
        C acc = C(2 * DIM) * C(u[idx]);
        if (p.i > 0) acc -= C(u[idx - 1]);
        if (p.i < n - 1) acc -= C(u[idx + 1]);
        if (p.j > 0) acc -= C(u[idx - sy]);
        if (p.j < n - 1) acc -= C(u[idx + sy]);
        if (DIM == 3) {
            if (p.k > 0) acc -= C(u[idx - sz]);
            if (p.k < n - 1) acc -= C(u[idx + sz]);
        }
        return C(op.s0) * acc;
    }
    C acc = C(op.D[idx]) * C(u[idx]);
    if (p.i > 0) acc -= C(op.ex[idx - 1]) * C(u[idx - 1]);
    if (p.i < n - 1) acc -= C(op.ex[idx]) * C(u[idx + 1]);
    if (p.j > 0) acc -= C(op.ey[idx - sy]) * C(u[idx - sy]);
    if (p.j < n - 1) acc -= C(op.ey[idx]) * C(u[idx + sy]);
    if (DIM == 3) {
        if (p.k > 0) acc -= C(op.ez[idx - sz]) * C(u[idx - sz]);
        if (p.k < n - 1) acc -= C(op.ez[idx]) * C(u[idx + sz]);
    }
    return acc;
}

// ----------------------------------------------------------- coarse operator

template <typename T>
struct CoarseOp {
    int n, N;
    const T* coef;   // 3^DIM * N
};

template <int DIM>
__host__ __device__ constexpr int stencil_points() { return DIM == 2 ? 9 : 27; }
template <int DIM>
__host__ __device__ constexpr int stencil_center() { return DIM == 2 ? 4 : 13; }

template <int DIM, typename C, typename T, typename F>
__device__ __forceinline__ C coarse_apply_fn(const CoarseOp<T>& op, int idx, const Idx<DIM>& p,
                                             F&& value_at) {
    const int n = op.n, N = op.N;
    C acc = C(0);
    int s = 0;
#pragma unroll
    for (int dz = (DIM == 3 ? -1 : 0); dz <= (DIM == 3 ? 1 : 0); ++dz) {
        const bool okz = (DIM == 2) || (p.k + dz >= 0 && p.k + dz < n);
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
            const bool oky = okz && p.j + dy >= 0 && p.j + dy < n;
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx, ++s) {
                const bool ok = oky && p.i + dx >= 0 && p.i + dx < n;
                if (ok) {
                    const int nb = idx + dx + n * (dy + n * dz);
                    acc += C(op.coef[(size_t)s * N + idx]) * value_at(nb);
                }
            }
        }
    }
    return acc;
}

// --------------------------------------------------------------- transfers

// One axis of linear interpolation at fine coordinate f (0-based): coarse
// node J sits on fine node 2J+1.  Returns up to two parents and weights.
struct Par {
    int lo, hi;
    float wlo, whi;
    int cnt;
};

__device__ __forceinline__ Par parents(int f, int nc) {
    Par q{0, 0, 0.f, 0.f, 0};
    if (f & 1) {                 // on coarse node (f-1)/2
        q.lo = (f - 1) >> 1;
        q.wlo = 1.f;
        q.cnt = 1;
        return q;
    }
    const int J = f >> 1;        // between coarse J-1 and J (boundary ones dropped)
    if (J >= 1) {
        q.lo = J - 1;
        q.wlo = 0.5f;
        q.cnt = 1;
    }
    if (J < nc) {
        if (q.cnt == 0) {
            q.lo = J;
            q.wlo = 0.5f;
            q.cnt = 1;
        } else {
            q.hi = J;
            q.whi = 0.5f;
            q.cnt = 2;
        }
    }
    return q;
}

// Interpolate one coarse column (values v, nc per axis) at fine node p.
template <int DIM, typename C, typename T>
__device__ __forceinline__ C interp_at(const T* __restrict__ v, int nc, const Idx<DIM>& p) {
    const Par px = parents(p.i, nc), py = parents(p.j, nc);
    C acc = C(0);
    if (DIM == 2) {
        for (int b = 0; b < py.cnt; ++b) {
            const int J = b ? py.hi : py.lo;
            const C wy = C(b ? py.whi : py.wlo);
            C rowv = C(0);
            for (int a = 0; a < px.cnt; ++a) {
                const int I = a ? px.hi : px.lo;
                rowv += C(a ? px.whi : px.wlo) * C(v[I + nc * J]);
            }
            acc += wy * rowv;
        }
    } else {
        const Par pz = parents(p.k, nc);
        for (int c = 0; c < pz.cnt; ++c) {
            const int K = c ? pz.hi : pz.lo;
            const C wz = C(c ? pz.whi : pz.wlo);
            C plane = C(0);
            for (int b = 0; b < py.cnt; ++b) {
                const int J = b ? py.hi : py.lo;
                const C wy = C(b ? py.whi : py.wlo);
                C rowv = C(0);
                for (int a = 0; a < px.cnt; ++a) {
                    const int I = a ? px.hi : px.lo;
                    rowv += C(a ? px.whi : px.wlo) * C(v[I + nc * (J + nc * K)]);
                }
                plane += wy * rowv;
            }
            acc += wz * plane;
        }
    }
    return acc;
}

// ------------------------------------------------------- row-mapped fine loop
//
// Fine-level kernels map work items to (x-row, i): each x-row of n nodes is
// padded to nxp = roundup(n, 64) items, so every wavefront lies inside one
// row and the row's (j, k) -- hence every y/z neighbour test and every y/z
// interpolation weight -- is uniform across the wavefront.  Lanes with
// i >= n idle.  The flat node index is i + n * row.
struct Rows {
    int n;       // nodes per axis
    int nxp;     // padded row length (multiple of 64)
    int total;   // rows * nxp
};

template <int DIM>
__device__ __forceinline__ bool row_item(const Rows& R, int w, Idx<DIM>& p, int& idx) {
    const int w0 = __builtin_amdgcn_readfirstlane(w);
    const int row = w0 / R.nxp;
    p.i = w - row * R.nxp;
    if (DIM == 2) {
        p.j = row;
        p.k = 0;
    } else {
        p.k = row / R.n;
        p.j = row - p.k * R.n;
    }
    const bool act = p.i < R.n;
    if (!act) p.i = R.n - 1;   // keep addresses in range on idle lanes
    idx = p.i + R.n * row;
    return act;
}

// Each block walks one contiguous range of rows (kBlock items at a time);
// with the XCD-aware logical block index, each XCD owns a contiguous slab.
__device__ __forceinline__ int row_chunk(int total) {
    const int per = (total + gridDim.x - 1) / gridDim.x;
    return (per + kBlock - 1) / kBlock * kBlock;
}

#define ROW_LOOP(R, lb)                                                                           \
    for (int c_ = row_chunk((R).total), w_ = (lb) * c_ + (int)threadIdx.x,                        \
             e_ = min((R).total, ((lb) + 1) * c_);                                                \
         w_ < e_; w_ += kBlock)

// Branch-free x-axis interpolation parents: two (possibly equal) coarse
// indices with weights (1, 0) on a coarse node, (1/2, 1/2) between two, and a
// zero weight for a boundary neighbour.
struct XPar {
    int lo, hi;
    float wlo, whi;
};

__device__ __forceinline__ XPar xparents(int f, int nc) {
    XPar q;
    if (f & 1) {
        q.lo = q.hi = (f - 1) >> 1;
        q.wlo = 1.f;
        q.whi = 0.f;
    } else {
        const int J = f >> 1;
        q.lo = J - 1;
        q.hi = J;
        q.wlo = q.whi = 0.5f;
        if (q.lo < 0) {
            q.lo = 0;
            q.wlo = 0.f;
        }
        if (q.hi >= nc) {
            q.hi = nc - 1;
            q.whi = 0.f;
        }
    }
    return q;
}

// Interpolate a coarse column at a fine node whose y/z parents are uniform.
template <int DIM, typename C, typename T>
__device__ __forceinline__ C interp_row(const T* __restrict__ v, int nc, const XPar& px, const Par& py,
                                        const Par& pz) {
    C acc = C(0);
    const int nzc = DIM == 3 ? pz.cnt : 1;
    for (int c = 0; c < nzc; ++c) {
        const int K = DIM == 3 ? (c ? pz.hi : pz.lo) : 0;
        const C wz = DIM == 3 ? C(c ? pz.whi : pz.wlo) : C(1);
        C plane = C(0);
        for (int b = 0; b < py.cnt; ++b) {
            const int J = b ? py.hi : py.lo;
            const C wy = C(b ? py.whi : py.wlo);
            const T* rowp = v + (size_t)nc * (J + (size_t)nc * K);
            const C rowv = C(px.wlo) * C(rowp[px.lo]) + C(px.whi) * C(rowp[px.hi]);
            plane += wy * rowv;
        }
        acc += wz * plane;
    }
    return acc;
}

// Level corrections at one fine node: z[c] for c < NB-1 interpolated from the
// NB-1 level-(L-1) columns, z[NB-1] = cL (the finest smoother output).
template <typename T>
struct ColPtrs {
    const T* p[kMaxNB];
};

template <int DIM, typename T, int NB>
__device__ __forceinline__ void fine_z(const ColPtrs<T>& Y, int nc, const T* __restrict__ cL, int idx,
                                       const Idx<DIM>& p, T (&z)[NB]) {
    if (NB > 1) {
        const XPar px = xparents(p.i, nc);
        const Par py = parents(p.j, nc);
        const Par pz = DIM == 3 ? parents(p.k, nc) : Par{0, 0, 1.f, 0.f, 1};
#pragma unroll
        for (int c = 0; c < NB - 1; ++c) z[c] = interp_row<DIM, T>(Y.p[c], nc, px, py, pz);
    }
    z[NB - 1] = cL[idx];
}

// ---------------------------------------------------------------- kernels

// r = b - A x (FP64), partial sums of ||b||^2 and ||r||^2.
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_init_residual(Rows R, FineOp<double> op, const double* __restrict__ b,
                                                          const double* __restrict__ x, double* __restrict__ r,
                                                          double* __restrict__ part) {
    const int lb = xcd_block(gridDim.x);
    double v[2] = {0.0, 0.0};
    ROW_LOOP(R, lb) {
        Idx<DIM> p;
        int idx;
        if (!row_item<DIM>(R, w_, p, idx)) continue;
        const double bi = b[idx];
        const double ri = bi - fine_apply<DIM, double>(op, x, idx, p);
        r[idx] = ri;
        v[0] += bi * bi;
        v[1] += ri * ri;
    }
    block_sum_store<2>(v, part, gridDim.x, lb);
}

// True-residual refresh r = b - A x in FP64 (mixed form, only when requested).
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_refresh(const Ctl* __restrict__ ctl, Rows R, FineOp<double> op,
                                                    const double* __restrict__ b, const double* __restrict__ x,
                                                    double* __restrict__ r, double* __restrict__ part) {
    if (ctl->state == 2 || !ctl->refresh_req) return;
    const int lb = xcd_block(gridDim.x);
    double v[1] = {0.0};
    ROW_LOOP(R, lb) {
        Idx<DIM> p;
        int idx;
        if (!row_item<DIM>(R, w_, p, idx)) continue;
        const double ri = b[idx] - fine_apply<DIM, double>(op, x, idx, p);
        r[idx] = ri;
        v[0] += ri * ri;
    }
    block_sum_store<1>(v, part, gridDim.x, lb);
}

// r -= Q alpha (pointwise, FP64 r), partial ||r||^2.
template <typename T, int NB>
__global__ void __launch_bounds__(kBlock) k_update_r(const Ctl* __restrict__ ctl, int N, const T* __restrict__ Q,
                                                     const double* __restrict__ alpha, double* __restrict__ r,
                                                     double* __restrict__ part) {
    if (ctl->state != 0) return;
    const int lb = xcd_block(gridDim.x);
    double a[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) a[c] = alpha[c];
    double v[1] = {0.0};
    for (int idx = lb * kBlock + threadIdx.x; idx < N; idx += gridDim.x * kBlock) {
        double ri = r[idx];
#pragma unroll
        for (int c = 0; c < NB; ++c) ri -= double(Q[(size_t)c * N + idx]) * a[c];
        r[idx] = ri;
        v[0] += ri * ri;
    }
    block_sum_store<1>(v, part, gridDim.x, lb);
}

// Fine-level damped Jacobi, first min(nu, 2) sweeps from c0 = 0:
//   c1 = omega (g / D);  c2 = c1 + omega ((g - A c1) / D)   (eq. (2)).
template <int DIM, typename T, typename G>
__global__ void __launch_bounds__(kBlock) k_fine_smooth(const Ctl* __restrict__ ctl, Rows R, FineOp<T> op,
                                                        const G* __restrict__ g, T* __restrict__ c, T omega,
                                                        int two_sweeps) {
    if (ctl->state != 0) return;
    const int lb = xcd_block(gridDim.x);
    const int n = op.n, sy = n, sz = n * n;
    ROW_LOOP(R, lb) {
        Idx<DIM> p;
        int idx;
        if (!row_item<DIM>(R, w_, p, idx)) continue;
        const T gi = T(g[idx]);
        const T Di = fine_diag<DIM>(op, idx);
        const T c1 = omega * (gi / Di);
        if (!two_sweeps) {
            c[idx] = c1;
            continue;
        }
        // A c1 with c1_j = omega (g_j / D_j) formed on the fly
        auto c1at = [&](int j) -> T { return omega * (T(g[j]) / fine_diag<DIM>(op, j)); };
        T Ac;
        if (!op.D) {
            T acc = T(2 * DIM) * c1;
            if (p.i > 0) acc -= c1at(idx - 1);
            if (p.i < n - 1) acc -= c1at(idx + 1);
            if (p.j > 0) acc -= c1at(idx - sy);
            if (p.j < n - 1) acc -= c1at(idx + sy);
            if (DIM == 3) {
                if (p.k > 0) acc -= c1at(idx - sz);
                if (p.k < n - 1) acc -= c1at(idx + sz);
            }
            Ac = op.s0 * acc;
        } else {
            T acc = Di * c1;
            if (p.i > 0) acc -= op.ex[idx - 1] * c1at(idx - 1);
            if (p.i < n - 1) acc -= op.ex[idx] * c1at(idx + 1);
            if (p.j > 0) acc -= op.ey[idx - sy] * c1at(idx - sy);
            if (p.j < n - 1) acc -= op.ey[idx] * c1at(idx + sy);
            if (DIM == 3) {
                if (p.k > 0) acc -= op.ez[idx - sz] * c1at(idx - sz);
                if (p.k < n - 1) acc -= op.ez[idx] * c1at(idx + sz);
            }
            Ac = acc;
        }
        c[idx] = c1 + omega * ((gi - Ac) / Di);
    }
}

// One further fine sweep: cout = cin + omega ((g - A cin) / D).
template <int DIM, typename T, typename G>
__global__ void __launch_bounds__(kBlock) k_fine_sweep(const Ctl* __restrict__ ctl, Rows R, FineOp<T> op,
                                                       const G* __restrict__ g, const T* __restrict__ cin,
                                                       T* __restrict__ cout, T omega) {
    if (ctl->state != 0) return;
    const int lb = xcd_block(gridDim.x);
    ROW_LOOP(R, lb) {
        Idx<DIM> p;
        int idx;
        if (!row_item<DIM>(R, w_, p, idx)) continue;
        const T res = T(g[idx]) - fine_apply<DIM, T>(op, cin, idx, p);
        cout[idx] = cin[idx] + omega * (res / fine_diag<DIM>(op, idx));
    }
}

// Full weighting g_c = 2^-d P^T g_f at every coarse node (thread per node).
template <int DIM, typename TI, typename TO>
__global__ void __launch_bounds__(kBlock) k_restrict(const Ctl* __restrict__ ctl, const TI* __restrict__ gf, int nf,
                                                     TO* __restrict__ gc, int nc, int Nc) {
    if (ctl->state != 0) return;
    const int idx = blockIdx.x * kBlock + threadIdx.x;
    if (idx >= Nc) return;
    const Idx<DIM> p = decomp<DIM>(idx, nc);
    using C = TO;
    C acc = C(0);
    const int fx = 2 * p.i + 1, fy = 2 * p.j + 1, fz = 2 * p.k + 1;
    for (int dz = (DIM == 3 ? -1 : 0); dz <= (DIM == 3 ? 1 : 0); ++dz) {
        const int z = fz + dz;
        if (DIM == 3 && z >= nf) continue;
        const C wz = (DIM == 3 && dz != 0) ? C(0.5) : C(1);
        C plane = C(0);
        for (int dy = -1; dy <= 1; ++dy) {
            const int y = fy + dy;
            if (y >= nf) continue;
            const C wy = dy ? C(0.5) : C(1);
            const size_t rowbase = (size_t)nf * (y + (DIM == 3 ? (size_t)nf * z : 0));
            C row = C(gf[rowbase + fx]);
            row += C(0.5) * C(gf[rowbase + fx - 1]);
            if (fx + 1 < nf) row += C(0.5) * C(gf[rowbase + fx + 1]);
            plane += wy * row;
        }
        acc += wz * plane;
    }
    gc[idx] = (DIM == 3 ? C(0.125) : C(0.25)) * acc;
}

// Level-fused damped Jacobi on all coarse levels in one launch: blocks
// [blk_off[l], blk_off[l+1]) smooth level l.  mode 0: first min(nu,2) sweeps
// from g (c1 formed on the fly); mode 1: one further sweep cin -> cout.
template <typename T>
struct CoarseLevels {
    int nlev;
    int blk_off[kMaxLevels + 1];
    int n[kMaxLevels];
    int N[kMaxLevels];
    const T* coef[kMaxLevels];
    const T* g[kMaxLevels];
    const T* cin[kMaxLevels];
    T* cout[kMaxLevels];
};

template <int DIM, typename T>
__global__ void __launch_bounds__(kBlock) k_coarse_smooth(const Ctl* __restrict__ ctl, CoarseLevels<T> L,
                                                          T omega, int mode, int two_sweeps) {
    if (ctl->state != 0) return;
    int l = 0;
    while (l + 1 < L.nlev && (int)blockIdx.x >= L.blk_off[l + 1]) ++l;
    const int idx = (blockIdx.x - L.blk_off[l]) * kBlock + threadIdx.x;
    const int N = L.N[l];
    if (idx >= N) return;
    CoarseOp<T> op{L.n[l], N, L.coef[l]};
    const T* __restrict__ g = L.g[l];
    const T* __restrict__ D = op.coef + (size_t)stencil_center<DIM>() * N;
    const Idx<DIM> p = decomp<DIM>(idx, op.n);
    const T gi = g[idx], Di = D[idx];
    if (mode == 0) {
        const T c1 = omega * (gi / Di);
        if (!two_sweeps) {
            L.cout[l][idx] = c1;
            return;
        }
        const T Ac = coarse_apply_fn<DIM, T>(op, idx, p, [&](int j) -> T { return omega * (g[j] / D[j]); });
        L.cout[l][idx] = c1 + omega * ((gi - Ac) / Di);
    } else {
        const T* __restrict__ cin = L.cin[l];
        const T Ac = coarse_apply_fn<DIM, T>(op, idx, p, [&](int j) -> T { return cin[j]; });
        L.cout[l][idx] = cin[idx] + omega * ((gi - Ac) / Di);
    }
}

// Prolongate ncols coarse columns to the next finer level (thread per fine node).

template <int DIM, typename T>
__global__ void __launch_bounds__(kBlock) k_prolong(const Ctl* __restrict__ ctl, ColPtrs<T> in, int ncols, int nc,
                                                    T* __restrict__ out, int nf, int Nf) {
    if (ctl->state != 0) return;
    const int idx = blockIdx.x * kBlock + threadIdx.x;
    if (idx >= Nf) return;
    const Idx<DIM> p = decomp<DIM>(idx, nf);
    for (int c = 0; c < ncols; ++c) out[(size_t)c * Nf + idx] = interp_at<DIM, T>(in.p[c], nc, p);
}

// W = Q_k^T Z_{k+1} partial sums (NB x NB, entry a*NB+c = Q column a . z^c).
template <int DIM, typename T, int NB>
__global__ void __launch_bounds__(kBlock) k_fine_W(const Ctl* __restrict__ ctl, Rows R, int N, ColPtrs<T> Y,
                                                   int nc, const T* __restrict__ cL, const T* __restrict__ Q,
                                                   double* __restrict__ part) {
    if (ctl->state != 0) return;
    const int lb = xcd_block(gridDim.x);
    double w[NB * NB];
#pragma unroll
    for (int q = 0; q < NB * NB; ++q) w[q] = 0.0;
    ROW_LOOP(R, lb) {
        Idx<DIM> p;
        int idx;
        if (!row_item<DIM>(R, w_, p, idx)) continue;
        T z[NB];
        fine_z<DIM, T, NB>(Y, nc, cL, idx, p, z);
#pragma unroll
        for (int a = 0; a < NB; ++a) {
            const double qa = double(Q[(size_t)a * N + idx]);
#pragma unroll
            for (int c = 0; c < NB; ++c) w[a * NB + c] += qa * double(z[c]);
        }
    }
    block_sum_store<NB * NB>(w, part, gridDim.x, lb);
}

// x += P_k alpha_k (deferred update of Algorithm 1); then, unless stopping,
// P_{k+1} = Z_{k+1} - P_k beta in place (Z recomputed from the coarse block).
// init = 1: P_0 = Z_0 only.
template <int DIM, typename T, int NB>
__global__ void __launch_bounds__(kBlock) k_update_xP(const Ctl* __restrict__ ctl, Rows R, int N, ColPtrs<T> Y,
                                                      int nc, const T* __restrict__ cL, T* __restrict__ P,
                                                      double* __restrict__ x, const double* __restrict__ alpha,
                                                      const double* __restrict__ beta, int init) {
    const int state = ctl->state;
    if (state == 2 || (init && state != 0)) return;
    const int lb = xcd_block(gridDim.x);
    __shared__ double sab[NB + NB * NB];
    if (!init) {
        for (int q = threadIdx.x; q < NB + NB * NB; q += kBlock) sab[q] = q < NB ? alpha[q] : beta[q - NB];
    }
    __syncthreads();
    ROW_LOOP(R, lb) {
        Idx<DIM> p;
        int idx;
        if (!row_item<DIM>(R, w_, p, idx)) continue;
        T pk[NB];
        if (!init) {
            double xi = x[idx];
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                pk[c] = P[(size_t)c * N + idx];
                xi += double(pk[c]) * sab[c];
            }
            x[idx] = xi;
            if (state != 0) continue;
        }
        T z[NB];
        fine_z<DIM, T, NB>(Y, nc, cL, idx, p, z);
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            double v = double(z[c]);
            if (!init) {
#pragma unroll
                for (int a2 = 0; a2 < NB; ++a2) v -= double(pk[a2]) * sab[NB + a2 * NB + c];
            }
            P[(size_t)c * N + idx] = T(v);
        }
    }
}

// Q = A P (block SpMM), partial sums of the Gram upper triangle P^T Q and of
// P^T r, value order [G_00, G_01, .., G_0,NB-1, G_11, .., G_NB-1,NB-1, g_0..g_NB-1].
template <int DIM, typename T, int NB>
__global__ void __launch_bounds__(kBlock) k_spmm_gram(const Ctl* __restrict__ ctl, Rows R, FineOp<T> op,
                                                      const T* __restrict__ P, T* __restrict__ Q,
                                                      const double* __restrict__ r, double* __restrict__ part) {
    if (ctl->state != 0) return;
    constexpr int NG = NB * (NB + 1) / 2;
    const int lb = xcd_block(gridDim.x);
    const int N = op.N;
    double acc[NG + NB];
#pragma unroll
    for (int q = 0; q < NG + NB; ++q) acc[q] = 0.0;
    ROW_LOOP(R, lb) {
        Idx<DIM> p;
        int idx;
        if (!row_item<DIM>(R, w_, p, idx)) continue;
        double pv[NB], qv[NB];
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            const T* Pc = P + (size_t)c * N;
            const T qc = fine_apply<DIM, T>(op, Pc, idx, p);
            Q[(size_t)c * N + idx] = qc;
            pv[c] = double(Pc[idx]);
            qv[c] = double(qc);
        }
        const double ri = r[idx];
        int q = 0;
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int c = a; c < NB; ++c) acc[q++] += pv[a] * qv[c];
#pragma unroll
        for (int a = 0; a < NB; ++a) acc[NG + a] += pv[a] * ri;
    }
    block_sum_store<NG + NB>(acc, part, gridDim.x, lb);
}

// Explicit Z (widened to double), for the mg_block entry point.
template <int DIM, typename T, int NB>
__global__ void __launch_bounds__(kBlock) k_write_Z(Rows R, int N, ColPtrs<T> Y, int nc, const T* __restrict__ cL,
                                                    double* __restrict__ Z) {
    ROW_LOOP(R, blockIdx.x) {
        Idx<DIM> p;
        int idx;
        if (!row_item<DIM>(R, w_, p, idx)) continue;
        T z[NB];
        fine_z<DIM, T, NB>(Y, nc, cL, idx, p, z);
#pragma unroll
        for (int c = 0; c < NB; ++c) Z[(size_t)c * N + idx] = double(z[c]);
    }
}

// b == 0: x = 0.
__global__ void __launch_bounds__(kBlock) k_zero_if(const Ctl* __restrict__ ctl, double* __restrict__ x, int N) {
    if (!ctl->zero_x) return;
    for (int idx = blockIdx.x * kBlock + threadIdx.x; idx < N; idx += gridDim.x * kBlock) x[idx] = 0.0;
}

}  // namespace amg
