// Structured-grid kernels of one MPCG iteration (Sec. 2, Algorithm 1).
//
// Layout in HBM (all levels): flat node index i + n*(j + n*k) (x fastest).
// Single vectors hold one value per node.  Blocks of several directions (the
// search block P, Q = A P, and the coarse block carry Y) are node-major: the
// S values of one node are contiguous, S = number of columns rounded up to
// even, so that one node's values move with paired (16-byte / 8-byte) loads.  Coarse operators are 3^d-point
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

#include <type_traits>

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
    T inv0;                // 1 / (2 dim h^-2) (constant coefficient), 1 / w9[4] (9-point)
    const T* iD;           // variable coefficient: 1 / diagonal (rounded once)
    int k9;                // 2D only: the operator is the constant 9-point stencil w9
    T w9[9];               // w9[(dy+1)*3 + (dx+1)] = A(idx, idx + dx + n dy)
};

template <int DIM, typename T>
__device__ __forceinline__ T fine_diag(const FineOp<T>& op, int idx) {
    if (DIM == 2 && op.k9) return op.w9[4];
    return op.D ? op.D[idx] : T(2 * DIM) * op.s0;
}

// sum_{dy,dx} w9 u(idx + dx + n dy) over the neighbours inside the grid
// (2D constant 9-point stencil), rows dy = -1, 0, 1 in turn.
template <typename C, typename T, typename F>
__device__ __forceinline__ C stencil9_apply(const FineOp<T>& op, int i, int j, int idx, F&& u) {
    // out-of-grid neighbours: weight 0 at the node's own address (loads
    // unconditional, the zero terms add exactly 0 in the same order)
    const int n = op.n;
    C acc = C(0);
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
        const bool oky = j + dy >= 0 && j + dy < n;
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            const bool ok = oky && i + dx >= 0 && i + dx < n;
            const C w = ok ? C(op.w9[(dy + 1) * 3 + dx + 1]) : C(0);
            acc += w * C(u(ok ? idx + dx + n * dy : idx));
        }
    }
    return acc;
}

// The 2*DIM face neighbours of a fine node in the order -x, +x, -y, +y, -z,
// +z: whether each lies inside the grid and its index, the node's own index
// when it does not (a valid address, so that neighbour loads need no
// branch: callers weight an outside neighbour by 0, which adds exactly 0).
template <int DIM>
struct FaceNbrs {
    bool ok[2 * DIM];
    int j[2 * DIM];
    int self;
    __device__ __forceinline__ FaceNbrs(const Idx<DIM>& p, int n, int idx) : self(idx) {
        const int sy = n, sz = n * n;
        ok[0] = p.i > 0;
        ok[1] = p.i < n - 1;
        ok[2] = p.j > 0;
        ok[3] = p.j < n - 1;
        j[0] = ok[0] ? idx - 1 : idx;
        j[1] = ok[1] ? idx + 1 : idx;
        j[2] = ok[2] ? idx - sy : idx;
        j[3] = ok[3] ? idx + sy : idx;
        if constexpr (DIM == 3) {
            ok[4] = p.k > 0;
            ok[5] = p.k < n - 1;
            j[4] = ok[4] ? idx - sz : idx;
            j[5] = ok[5] ? idx + sz : idx;
        }
    }
    // Face coefficient between the node and neighbour q, stored at the lower
    // node of the face: the neighbour for -x/-y/-z, the node itself for
    // +x/+y/+z (for an outside neighbour a valid address, weighted 0).
    template <typename Op>
    __device__ __forceinline__ auto face(const Op& op, int q) const {
        const auto* e = q < 2 ? op.ex : (q < 4 ? op.ey : op.ez);
        return e[(q & 1) ? self : j[q]];
    }
};

// 1 / D, precomputed: the smoother multiplies by it instead of dividing.
template <int DIM, typename T>
__device__ __forceinline__ T fine_invdiag(const FineOp<T>& op, int idx) {
    return op.iD ? op.iD[idx] : op.inv0;
}

// (A u)_idx on the finest level, computed in type C.
template <int DIM, typename C, typename T, typename U>
__device__ __forceinline__ C fine_apply(const FineOp<T>& op, const U* __restrict__ u, int idx,
                                        const Idx<DIM>& p) {
    const int n = op.n;
    const int sy = n, sz = n * n;
    if (DIM == 2 && op.k9) return stencil9_apply<C, T>(op, p.i, p.j, idx, [&](int q) { return u[q]; });
    const FaceNbrs<DIM> f(p, n, idx);
    if (!op.D) {
        C acc = C(2 * DIM) * C(u[idx]);
#pragma unroll
        for (int q = 0; q < 2 * DIM; ++q) acc -= (f.ok[q] ? C(1) : C(0)) * C(u[f.j[q]]);
        return C(op.s0) * acc;
    }
    C acc = C(op.D[idx]) * C(u[idx]);
#pragma unroll
    for (int q = 0; q < 2 * DIM; ++q) acc -= (f.ok[q] ? C(f.face(op, q)) : C(0)) * C(u[f.j[q]]);
    return acc;
}

// ----------------------------------------------------------- coarse operator

template <typename T>
struct CoarseOp {
    int n, N;
    const T* coef;   // 3^DIM * N, or (cst) the 3^DIM values of a constant stencil
    int cst;         // 1: every node has the same stencil, truncated at the boundary
};

template <int DIM>
__host__ __device__ constexpr int stencil_points() { return DIM == 2 ? 9 : 27; }
template <int DIM>
__host__ __device__ constexpr int stencil_center() { return DIM == 2 ? 4 : 13; }

// The 3^d taps of a coarse stencil at node idx, weight(s) giving tap s.  A
// neighbour outside the grid takes weight 0 and the node's own (valid)
// address, so every load is unconditional and all of them issue at once (a
// load under a divergent branch waits for the one before it); the zero
// terms add exactly 0 in the same summation order.
template <int DIM, typename C, typename W, typename F>
__device__ __forceinline__ C coarse_taps(int n, int idx, const Idx<DIM>& p, W&& weight, F&& value_at) {
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
                const int nb = ok ? idx + dx + n * (dy + n * dz) : idx;
                const C w = C(weight(s));
                acc += (ok ? w : C(0)) * value_at(nb);
            }
        }
    }
    return acc;
}

// A_l applied at node idx.  The constant-stencil branch is taken per level
// (uniform), so its 3^d weights are read once per wave through scalar loads
// rather than once per lane and tap.
template <int DIM, typename C, typename T, typename F>
__device__ __forceinline__ C coarse_apply_fn(const CoarseOp<T>& op, int idx, const Idx<DIM>& p,
                                             F&& value_at) {
    const T* __restrict__ coef = op.coef;
    if (op.cst) return coarse_taps<DIM, C>(op.n, idx, p, [&](int s) -> T { return coef[s]; }, value_at);
    const int N = op.N;
    return coarse_taps<DIM, C>(op.n, idx, p, [&](int s) -> T { return coef[(size_t)s * N + idx]; }, value_at);
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

// ------------------------------------------------------------ vector access

template <typename T>
struct Pair;
template <>
struct Pair<double> {
    using type = double2;
};
template <>
struct Pair<float> {
    using type = float2;
};

// Columns rounded up to even: the node stride of a block.
__host__ __device__ constexpr int even_up(int k) { return k + (k & 1); }

template <typename T, int S>
__device__ __forceinline__ void load_node(const T* __restrict__ p, T (&o)[S]) {
    static_assert(S % 2 == 0, "node stride must be even");
    const typename Pair<T>::type* q = reinterpret_cast<const typename Pair<T>::type*>(p);
#pragma unroll
    for (int c = 0; c < S / 2; ++c) {
        const typename Pair<T>::type v = q[c];
        o[2 * c] = v.x;
        o[2 * c + 1] = v.y;
    }
}

template <typename T, int S>
__device__ __forceinline__ void store_node(T* __restrict__ p, const T (&o)[S]) {
    typename Pair<T>::type* q = reinterpret_cast<typename Pair<T>::type*>(p);
#pragma unroll
    for (int c = 0; c < S / 2; ++c) {
        typename Pair<T>::type v;
        v.x = o[2 * c];
        v.y = o[2 * c + 1];
        q[c] = v;
    }
}

// Store the node-major values o of the wavefront's 64 consecutive nodes
// (lane l: node l of the range starting at dst; lanes >= nact store nothing)
// as whole-wavefront runs: the values pass through the wavefront's LDS slice
// buf (64 S values), then store q writes bytes [q * 64 PB, (q + 1) * 64 PB) of
// the range, PB bytes per lane, instead of each lane writing its own node's
// bytes at a 64-node stride (three times the L2 write requests for 48-byte
// nodes).  All 64 lanes must call it; dst must be PB-aligned.
template <typename T, int S>
__device__ __forceinline__ void store_nodes_wave(T* __restrict__ dst, int nact, T* buf, const T (&o)[S]) {
    constexpr int NBYTES = S * (int)sizeof(T);
    constexpr int PB = NBYTES % 16 == 0 ? 16 : 8;   // bytes per lane and store
    constexpr int NP = NBYTES / PB;                 // stores per wavefront
    using Piece = typename std::conditional<PB == 16, int4, int2>::type;
    const int lane = threadIdx.x & 63;
    store_node<T, S>(buf + lane * S, o);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const Piece* src = reinterpret_cast<const Piece*>(buf);
    Piece* d = reinterpret_cast<Piece*>(dst);
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        const int pc = q * 64 + lane;
        if (pc < nact * NP) d[pc] = src[pc];
    }
    // the slice is free again once every lane has read its pieces
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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

// The unclamped x index of item w in its row (lanes past the row end
// included).
__device__ __forceinline__ int row_x(const Rows& R, int w) {
    const int w0 = __builtin_amdgcn_readfirstlane(w);
    return w - (w0 / R.nxp) * R.nxp;
}

// Each XCD (blocks b with the same b % 8) owns one contiguous slab of the
// rows, and its blocks walk the slab together, kBlock items per block and
// step, block j of the XCD taking the j-th kBlock items of each step's band.
// The XCD's resident blocks thus cover a thin band of consecutive rows at a
// time, so the +-y and +-z neighbours (and coarse interpolation parents) a
// kernel reads were fetched shortly before by a block of the same XCD and
// are still in that XCD's L2.  Grids whose size is not a multiple of 8 walk
// the whole range as one slab.
struct Band {
    int start, end, stride;
};

// The band of block bid in a walk by g blocks (a launch's own blocks, or a
// block range of a launch that starts at a multiple of 8, which keeps every
// block on the XCD its index names).
__device__ __forceinline__ Band row_band_of(int total, int bid, int g) {
    const int x = (g % kNumXcd) ? 0 : bid % kNumXcd;
    const int nb = (g % kNumXcd) ? g : g / kNumXcd;
    const int j = (g % kNumXcd) ? bid : bid / kNumXcd;
    const int slabs = (g % kNumXcd) ? 1 : kNumXcd;
    const int per = ((total + slabs - 1) / slabs + kBlock - 1) / kBlock * kBlock;
    Band b;
    b.start = x * per + j * kBlock + (int)threadIdx.x;
    b.end = min(total, (x + 1) * per);
    b.stride = nb * kBlock;
    return b;
}

__device__ __forceinline__ Band row_band(int total) { return row_band_of(total, (int)blockIdx.x, (int)gridDim.x); }

// lb: the block's index for its reduction partials (unused by the walk).
#define ROW_LOOP(R, lb)                                                                           \
    for (Band b_ = row_band((R).total), *bp_ = &b_; bp_; bp_ = nullptr)                            \
        for (int w_ = b_.start; w_ < b_.end; w_ += b_.stride)

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

// Interpolate all S columns of a node-major coarse block (stride S) at a fine
// node; the y/z parents are uniform across the wavefront.
template <int DIM, typename T, int S, typename Node>
__device__ __forceinline__ void interp_block_fn(Node&& node, const XPar& px, const Par& py, const Par& pz,
                                                T (&z)[S]) {
    // Two parents per axis always: a missing second parent takes weight 0
    // and the first one's address, so all node loads are unconditional and
    // issue together; the zero terms add exactly 0 in the same order.
#pragma unroll
    for (int c = 0; c < S; ++c) z[c] = T(0);
    constexpr int nzc = DIM == 3 ? 2 : 1;
#pragma unroll
    for (int cz = 0; cz < nzc; ++cz) {
        const bool zlo = cz == 0 || pz.cnt < 2;
        const int K = DIM == 3 ? (zlo ? pz.lo : pz.hi) : 0;
        const T wz = DIM == 3 ? (cz == 0 ? T(pz.wlo) : (pz.cnt < 2 ? T(0) : T(pz.whi))) : T(1);
        T plane[S];
#pragma unroll
        for (int c = 0; c < S; ++c) plane[c] = T(0);
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const bool ylo = b == 0 || py.cnt < 2;
            const int J = ylo ? py.lo : py.hi;
            const T wy = b == 0 ? T(py.wlo) : (py.cnt < 2 ? T(0) : T(py.whi));
            T lo[S], hi[S];
            node(px.lo, J, K, lo);
            node(px.hi, J, K, hi);
#pragma unroll
            for (int c = 0; c < S; ++c) plane[c] += wy * (T(px.wlo) * lo[c] + T(px.whi) * hi[c]);
        }
#pragma unroll
        for (int c = 0; c < S; ++c) z[c] += wz * plane[c];
    }
}

// Interpolation of a node-major coarse block Y (S values per node).
template <int DIM, typename T, int S>
__device__ __forceinline__ void interp_block(const T* __restrict__ Y, int nc, const XPar& px, const Par& py,
                                             const Par& pz, T (&z)[S]) {
    interp_block_fn<DIM, T, S>(
        [&](int I, int J, int K, T (&o)[S]) { load_node<T, S>(Y + ((size_t)nc * (J + (size_t)nc * K) + I) * S, o); },
        px, py, pz, z);
}

// Directions at one fine node: the NB - NE level corrections, z[c] for
// c < NB-NE-1 interpolated from the node-major level-(L-1) block Y (stride
// even_up(NB-NE-1)) and z[NB-NE-1] = cL (the finest smoother output); with
// NE = 1 the learned direction z[NB-1] = dl[idx] (0 when dzero: a non-finite
// network output gives a zero column).
template <int DIM, typename T, int NB, int NE>
__device__ __forceinline__ void fine_z(const T* __restrict__ Y, int nc, const T* __restrict__ cL,
                                       const T* __restrict__ dl, bool dzero, int idx, const Idx<DIM>& p,
                                       T (&z)[NB]) {
    constexpr int NL = NB - NE;
    if (NL > 1) {
        constexpr int SY = even_up(NL > 1 ? NL - 1 : 1);
        const XPar px = xparents(p.i, nc);
        const Par py = parents(p.j, nc);
        const Par pz = DIM == 3 ? parents(p.k, nc) : Par{0, 0, 1.f, 0.f, 1};
        T zy[SY];
        interp_block<DIM, T, SY>(Y, nc, px, py, pz, zy);
#pragma unroll
        for (int c = 0; c < NL - 1; ++c) z[c] = zy[c];
    }
    z[NL - 1] = cL[idx];
    if (NE) z[NB - 1] = dzero ? T(0) : dl[idx];
}

template <int DIM, typename T, int NB, int NE>
struct ZWave {
    static constexpr int NL = NB - NE;
    static constexpr int SY = even_up(NL > 1 ? NL - 1 : 1);
    static constexpr int NZC = DIM == 3 ? 2 : 1;
    T v[NL > 1 ? NZC : 1][2][NL > 1 ? SY : 1];   // coarse parents: [z][y][column]
    T cl, dlv;                                  // cL and the learned direction at the node
};

// Load phase: every load of fine_z_wave, issued without waiting on any of
// them (the branches around them are uniform or lane masks), so that a
// caller can issue its own loads beside them and wait once.  Lanes 0..32
// load the coarse parents (outside the grid at a clamped node); a missing
// second y or z parent is not loaded but set to zero (weight 0 in the
// combine phase).
template <int DIM, typename T, int NB, int NE>
__device__ __forceinline__ void fine_z_wave_load(const T* __restrict__ Y, int nc, const T* __restrict__ cL,
                                                 const T* __restrict__ dl, int idx, const Idx<DIM>& p, int i_row,
                                                 ZWave<DIM, T, NB, NE>& zw) {
    using ZW = ZWave<DIM, T, NB, NE>;
    zw.cl = cL[idx];
    zw.dlv = NE ? dl[idx] : T(0);
    if constexpr (ZW::NL > 1) {
        const int lane = threadIdx.x & 63;
        const int i0 = __builtin_amdgcn_readfirstlane(i_row);
        const int Jc = min(max((i0 >> 1) - 1 + lane, 0), nc - 1);
        const Par py = parents(p.j, nc);
        const Par pz = DIM == 3 ? parents(p.k, nc) : Par{0, 0, 1.f, 0.f, 1};
#pragma unroll
        for (int cz = 0; cz < ZW::NZC; ++cz)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int c = 0; c < ZW::SY; ++c) zw.v[cz][b][c] = T(0);
        if (lane <= 32) {
#pragma unroll
            for (int cz = 0; cz < ZW::NZC; ++cz) {
                if (cz == 1 && pz.cnt < 2) continue;
                const int K = DIM == 3 ? (cz == 0 ? pz.lo : pz.hi) : 0;
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    if (b == 1 && py.cnt < 2) continue;
                    const int Jy = b == 0 ? py.lo : py.hi;
                    load_node<T, ZW::SY>(Y + ((size_t)nc * (Jy + (size_t)nc * K) + Jc) * ZW::SY, zw.v[cz][b]);
                }
            }
        }
    }
}

// Combine phase (all 64 lanes): the y/z weights per coarse x parent, then
// each fine lane's two x parents by shuffles; the zero-weight terms add
// exactly 0.
template <int DIM, typename T, int NB, int NE>
__device__ __forceinline__ void fine_z_wave_finish(const ZWave<DIM, T, NB, NE>& zw, int nc, bool dzero,
                                                   const Idx<DIM>& p, int i_row, T (&z)[NB]) {
    using ZW = ZWave<DIM, T, NB, NE>;
    constexpr int NL = ZW::NL;
    if constexpr (NL > 1) {
        constexpr int SY = ZW::SY;
        const int lane = threadIdx.x & 63;
        const int i0 = __builtin_amdgcn_readfirstlane(i_row);
        const int jb = (i0 >> 1) - 1;
        const int J = jb + lane;
        const bool jin = lane <= 32 && J >= 0 && J < nc;
        const Par py = parents(p.j, nc);
        const Par pz = DIM == 3 ? parents(p.k, nc) : Par{0, 0, 1.f, 0.f, 1};
        T row[SY];
#pragma unroll
        for (int c = 0; c < SY; ++c) row[c] = T(0);
#pragma unroll
        for (int cz = 0; cz < ZW::NZC; ++cz) {
            const T wz = DIM == 3 ? (cz == 0 ? T(pz.wlo) : (pz.cnt < 2 ? T(0) : T(pz.whi))) : T(1);
            T plane[SY];
#pragma unroll
            for (int c = 0; c < SY; ++c) plane[c] = T(0);
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const T wy = b == 0 ? T(py.wlo) : (py.cnt < 2 ? T(0) : T(py.whi));
#pragma unroll
                for (int c = 0; c < SY; ++c) plane[c] += wy * zw.v[cz][b][c];
            }
#pragma unroll
            for (int c = 0; c < SY; ++c) row[c] += wz * plane[c];
        }
#pragma unroll
        for (int c = 0; c < SY; ++c) row[c] = jin ? row[c] : T(0);
        const XPar px = xparents(p.i, nc);
        const int llo = min(max(px.lo - jb, 0), 32), lhi = min(max(px.hi - jb, 0), 32);
#pragma unroll
        for (int c = 0; c < NL - 1; ++c) {
            const T a = __shfl(row[c], llo);
            const T b2 = __shfl(row[c], lhi);
            z[c] = T(px.wlo) * a + T(px.whi) * b2;
        }
    }
    z[NL - 1] = zw.cl;
    if (NE) z[NB - 1] = dzero ? T(0) : zw.dlv;
}

// fine_z for a whole wavefront (all 64 lanes must call it; lanes past the
// row end use a clamped node and their result is discarded).  The wave's 64
// fine nodes lie in one x-row, so their y/z parents are common and their x
// parents are 33 consecutive coarse nodes: lane l (< 33) first combines the
// y/z parents at coarse x = i0/2 - 1 + l into one value per column, and each
// fine lane then takes its two x parents from those lanes by shuffles.  Per
// fine node that is a quarter of the coarse loads of fine_z.
template <int DIM, typename T, int NB, int NE>
__device__ __forceinline__ void fine_z_wave(const T* __restrict__ Y, int nc, const T* __restrict__ cL,
                                            const T* __restrict__ dl, bool dzero, int idx, const Idx<DIM>& p,
                                            int i_row, T (&z)[NB]) {
    ZWave<DIM, T, NB, NE> zw;
    fine_z_wave_load<DIM, T, NB, NE>(Y, nc, cL, dl, idx, p, i_row, zw);
    fine_z_wave_finish<DIM, T, NB, NE>(zw, nc, dzero, p, i_row, z);
}

// (A P)_idx for all columns of a node-major block on the finest level.
template <int DIM, typename T, int S>
__device__ __forceinline__ void fine_apply_block(const FineOp<T>& op, const T* __restrict__ P, int idx,
                                                 const Idx<DIM>& p, T (&own)[S], T (&q)[S]) {
    const int n = op.n, sy = n, sz = n * n;
    load_node<T, S>(P + (size_t)idx * S, own);
    T nb[S];
    if (DIM == 2 && op.k9) {
#pragma unroll
        for (int c = 0; c < S; ++c) q[c] = T(0);
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
            if (p.j + dy < 0 || p.j + dy >= n) continue;
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                if (p.i + dx < 0 || p.i + dx >= n) continue;
                const T w = op.w9[(dy + 1) * 3 + dx + 1];
                load_node<T, S>(P + (size_t)(idx + dx + n * dy) * S, nb);
#pragma unroll
                for (int c = 0; c < S; ++c) q[c] += w * nb[c];
            }
        }
        return;
    }
    if (!op.D) {
#pragma unroll
        for (int c = 0; c < S; ++c) q[c] = T(2 * DIM) * own[c];
        auto sub = [&](int j) {
            load_node<T, S>(P + (size_t)j * S, nb);
#pragma unroll
            for (int c = 0; c < S; ++c) q[c] -= nb[c];
        };
        if (p.i > 0) sub(idx - 1);
        if (p.i < n - 1) sub(idx + 1);
        if (p.j > 0) sub(idx - sy);
        if (p.j < n - 1) sub(idx + sy);
        if (DIM == 3) {
            if (p.k > 0) sub(idx - sz);
            if (p.k < n - 1) sub(idx + sz);
        }
#pragma unroll
        for (int c = 0; c < S; ++c) q[c] *= op.s0;
        return;
    }
    const T d = op.D[idx];
#pragma unroll
    for (int c = 0; c < S; ++c) q[c] = d * own[c];
    auto sub = [&](int j, T e) {
        load_node<T, S>(P + (size_t)j * S, nb);
#pragma unroll
        for (int c = 0; c < S; ++c) q[c] -= e * nb[c];
    };
    if (p.i > 0) sub(idx - 1, op.ex[idx - 1]);
    if (p.i < n - 1) sub(idx + 1, op.ex[idx]);
    if (p.j > 0) sub(idx - sy, op.ey[idx - sy]);
    if (p.j < n - 1) sub(idx + sy, op.ey[idx]);
    if (DIM == 3) {
        if (p.k > 0) sub(idx - sz, op.ez[idx - sz]);
        if (p.k < n - 1) sub(idx + sz, op.ez[idx]);
    }
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

// y = A x on the finest level in FP64.
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_apply(Rows R, FineOp<double> op, const double* __restrict__ x,
                                                  double* __restrict__ y) {
    ROW_LOOP(R, blockIdx.x) {
        Idx<DIM> p;
        int idx;
        if (!row_item<DIM>(R, w_, p, idx)) continue;
        y[idx] = fine_apply<DIM, double>(op, x, idx, p);
    }
}

// w = Q^T d partial sums (Q node-major, NB columns, stride even_up(NB)).
template <typename T, int NB>
__global__ void __launch_bounds__(kBlock) k_cols_dot(const T* __restrict__ Q, const double* __restrict__ d, int N,
                                                     double* __restrict__ part) {
    constexpr int S = even_up(NB);
    double w[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) w[c] = 0.0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < N; i += gridDim.x * kBlock) {
        T q[S];
        load_node<T, S>(Q + (size_t)i * S, q);
        const double di = d[i];
#pragma unroll
        for (int c = 0; c < NB; ++c) w[c] += double(q[c]) * di;
    }
    block_sum_store<NB>(w, part, gridDim.x, blockIdx.x);
}

// t = G^+ w with w reduced from the k_cols_dot partials (one block).
template <int NB>
__global__ void __launch_bounds__(kRedBlock) k_proj_coef(const double* __restrict__ part, int nblk,
                                                         const double* __restrict__ Gplus, double* __restrict__ t) {
    __shared__ double w[NB];
    reduce_partials<NB>(part, nblk, w);
    if (threadIdx.x < NB) {
        double s = 0.0;
        for (int m = 0; m < NB; ++m) s += Gplus[threadIdx.x * NB + m] * w[m];
        t[threadIdx.x] = s;
    }
}

// out = q - Q t (Q node-major).
template <typename T, int NB>
__global__ void __launch_bounds__(kBlock) k_sub_cols(const double* __restrict__ q, const T* __restrict__ Q,
                                                     const double* __restrict__ t, double* __restrict__ out, int N) {
    constexpr int S = even_up(NB);
    __shared__ double ts[NB];
    if (threadIdx.x < NB) ts[threadIdx.x] = t[threadIdx.x];
    __syncthreads();
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < N; i += gridDim.x * kBlock) {
        T qq[S];
        load_node<T, S>(Q + (size_t)i * S, qq);
        double v = q[i];
#pragma unroll
        for (int c = 0; c < NB; ++c) v -= double(qq[c]) * ts[c];
        out[i] = v;
    }
}

// Training pair of the learned direction: r = b - A x (FP64) and e = xs - x.
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_pair(Rows R, FineOp<double> op, const double* __restrict__ b,
                                                 const double* __restrict__ xs, const double* __restrict__ x,
                                                 double* __restrict__ r, double* __restrict__ e) {
    ROW_LOOP(R, blockIdx.x) {
        Idx<DIM> p;
        int idx;
        if (!row_item<DIM>(R, w_, p, idx)) continue;
        r[idx] = b[idx] - fine_apply<DIM, double>(op, x, idx, p);
        e[idx] = xs[idx] - x[idx];
    }
}

// r -= Q alpha (pointwise, FP64 r; Q node-major), partial ||r||^2.
template <typename T, int NB>
__global__ void __launch_bounds__(kBlock) k_update_r(const Ctl* __restrict__ ctl, int N, const T* __restrict__ Q,
                                                     const double* __restrict__ alpha, double* __restrict__ r,
                                                     double* __restrict__ part) {
    if (ctl->state != 0) return;
    constexpr int S = even_up(NB);
    const int lb = xcd_block(gridDim.x);
    double a[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) a[c] = alpha[c];
    double v[1] = {0.0};
    const int per = ((N + gridDim.x - 1) / gridDim.x + kBlock - 1) / kBlock * kBlock;
    const int end = min(N, (lb + 1) * per);
    for (int idx = lb * per + threadIdx.x; idx < end; idx += kBlock) {
        T q[S];
        load_node<T, S>(Q + (size_t)idx * S, q);
        double ri = r[idx];
#pragma unroll
        for (int c = 0; c < NB; ++c) ri -= double(q[c]) * a[c];
        r[idx] = ri;
        v[0] += ri * ri;
    }
    block_sum_store<1>(v, part, gridDim.x, lb);
}

// Fine-level damped Jacobi at one node, first min(nu, 2) sweeps from c0 = 0:
//   c1 = omega (g / D);  c2 = c1 + omega ((g - A c1) / D)   (eq. (2)).
template <int DIM, typename T, typename G>
__device__ __forceinline__ T fine_smooth_at(const FineOp<T>& op, const G* __restrict__ g, int idx, const Idx<DIM>& p,
                                            T omega, int two_sweeps) {
    const int n = op.n, sy = n, sz = n * n;
    if (!two_sweeps || (DIM == 2 && op.k9)) {
        const T gi = T(g[idx]);
        const T iDi = fine_invdiag<DIM>(op, idx);
        const T c1 = omega * (gi * iDi);
        if (!two_sweeps) return c1;
        // A c1 with c1_j = omega g_j / D_j formed on the fly
        auto c1at = [&](int j) -> T { return omega * (T(g[j]) * fine_invdiag<DIM>(op, j)); };
        const T Ac = stencil9_apply<T, T>(op, p.i, p.j, idx, c1at);
        return c1 + omega * ((gi - Ac) * iDi);
    }
    // face stencil, two sweeps: every load first (g at the node and its face
    // neighbours at clamped indices, then 1/D and the coefficients when they
    // vary; the branches on them are uniform), then the arithmetic
    const FaceNbrs<DIM> f(p, n, idx);
    const T gi = T(g[idx]);
    T gq[2 * DIM], iq[2 * DIM], fq[2 * DIM];
#pragma unroll
    for (int q = 0; q < 2 * DIM; ++q) gq[q] = T(g[f.j[q]]);
    T iDi = op.inv0, Dd = T(0);
#pragma unroll
    for (int q = 0; q < 2 * DIM; ++q) iq[q] = op.inv0;
    if (op.iD) {
        iDi = op.iD[idx];
#pragma unroll
        for (int q = 0; q < 2 * DIM; ++q) iq[q] = op.iD[f.j[q]];
    }
    if (op.D) {
        Dd = op.D[idx];
#pragma unroll
        for (int q = 0; q < 2 * DIM; ++q) fq[q] = f.face(op, q);
    }
    // A c1 with c1_j = omega g_j / D_j
    const T c1 = omega * (gi * iDi);
    T Ac;
    if (!op.D) {
        T acc = T(2 * DIM) * c1;
#pragma unroll
        for (int q = 0; q < 2 * DIM; ++q) acc -= (f.ok[q] ? T(1) : T(0)) * (omega * (gq[q] * iq[q]));
        Ac = op.s0 * acc;
    } else {
        T acc = Dd * c1;
#pragma unroll
        for (int q = 0; q < 2 * DIM; ++q) acc -= (f.ok[q] ? fq[q] : T(0)) * (omega * (gq[q] * iq[q]));
        Ac = acc;
    }
    return c1 + omega * ((gi - Ac) * iDi);
}

template <int DIM, typename T, typename G>
__global__ void __launch_bounds__(kBlock) k_fine_smooth(const Ctl* __restrict__ ctl, Rows R, FineOp<T> op,
                                                        const G* __restrict__ g, T* __restrict__ c, T omega,
                                                        int two_sweeps) {
    if (ctl->state != 0) return;
    const int lb = xcd_block(gridDim.x);
    ROW_LOOP(R, lb) {
        Idx<DIM> p;
        int idx;
        if (!row_item<DIM>(R, w_, p, idx)) continue;
        c[idx] = fine_smooth_at<DIM, T, G>(op, g, idx, p, omega, two_sweeps);
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
        cout[idx] = cin[idx] + omega * (res * fine_invdiag<DIM>(op, idx));
    }
}

// Full weighting g_c = 2^-d P^T g_f at coarse node idx (coarse node J on
// fine node 2J+1; weights 1, 1/2 per axis, boundary neighbours dropped).
template <int DIM, typename TI, typename C>
__device__ __forceinline__ C restrict_at(const TI* __restrict__ gf, int nf, int nc, int idx) {
    const Idx<DIM> p = decomp<DIM>(idx, nc);
    // per axis: fine 2J, 2J+1, 2J+2 with weights 1/2, 1, 1/2; a node past the
    // grid gets weight 0 and a clamped (valid) address, so all loads issue at once
    const int fx = 2 * p.i, fy = 2 * p.j, fz = 2 * p.k;
    const C w2x = fx + 2 < nf ? C(0.5) : C(0), w2y = fy + 2 < nf ? C(0.5) : C(0);
    const int x2 = min(fx + 2, nf - 1), y2 = min(fy + 2, nf - 1);
    const int ys[3] = {fy, fy + 1, y2};
    const C wy[3] = {C(0.5), C(1), w2y};
    C acc = C(0);
    const int nzs = DIM == 3 ? 3 : 1;
    const C w2z = DIM == 3 && fz + 2 < nf ? C(0.5) : C(0);
    const int zs[3] = {fz, fz + 1, min(fz + 2, nf - 1)};
    const C wz[3] = {C(0.5), C(1), w2z};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (a >= nzs) break;
        const size_t zb = DIM == 3 ? (size_t)nf * nf * zs[a] : 0;
        C plane = C(0);
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const TI* rowp = gf + zb + (size_t)nf * ys[b];
            const C row = C(0.5) * C(rowp[fx]) + C(rowp[fx + 1]) + w2x * C(rowp[x2]);
            plane += wy[b] * row;
        }
        acc += (DIM == 3 ? wz[a] : C(1)) * plane;
    }
    return (DIM == 3 ? C(0.125) : C(0.25)) * acc;
}

// Restriction to one coarse level (thread per coarse node).  Also writes the
// first Jacobi sweep c1 = omega (g / D) of that level (read by the smoother).
// dconst: D is the one diagonal value of a constant stencil.
template <int DIM, typename TI, typename TO>
__global__ void __launch_bounds__(kBlock) k_restrict(const Ctl* __restrict__ ctl, const TI* __restrict__ gf, int nf,
                                                     TO* __restrict__ gc, int nc, int Nc, const TO* __restrict__ D,
                                                     TO* __restrict__ c1, TO omega, int dconst) {
    if (ctl->state != 0) return;
    const int idx = blockIdx.x * kBlock + threadIdx.x;
    if (idx >= Nc) return;
    const TO g = restrict_at<DIM, TI, TO>(gf, nf, nc, idx);
    gc[idx] = g;
    c1[idx] = omega * (g / D[dconst ? 0 : idx]);
}

// The small coarse levels of the restriction chain in one block, one level
// after the other.
template <typename T>
struct RestrictChain {
    int count;
    int nf[kMaxLevels], nc[kMaxLevels], Nc[kMaxLevels];
    const T* gf[kMaxLevels];
    T* gc[kMaxLevels];
    const T* D[kMaxLevels];
    T* c1[kMaxLevels];
    int dconst[kMaxLevels];   // D is one value (constant stencil)
};

constexpr int kTailBlock = 1024;

template <int DIM, typename T>
__global__ void __launch_bounds__(kTailBlock) k_restrict_tail(const Ctl* __restrict__ ctl, RestrictChain<T> ch,
                                                              T omega) {
    if (ctl->state != 0) return;
    for (int m = 0; m < ch.count; ++m) {
        for (int idx = threadIdx.x; idx < ch.Nc[m]; idx += kTailBlock) {
            const T g = restrict_at<DIM, T, T>(ch.gf[m], ch.nf[m], ch.nc[m], idx);
            ch.gc[m][idx] = g;
            ch.c1[m][idx] = omega * (g / ch.D[m][ch.dconst[m] ? 0 : idx]);
        }
        __syncthreads();
    }
}

// Level-fused damped Jacobi on all coarse levels in one launch: blocks
// [blk_off[l], blk_off[l+1]) smooth level l.  mode 0: first min(nu,2) sweeps
// from g (c1 formed on the fly); mode 1: one further sweep cin -> cout.
// The output of level l goes to cout[l][idx * cstride[l]] (the last column
// of the node-major block carry after the final sweep).
template <typename T>
struct CoarseLevels {
    int nlev;
    int blk_off[kMaxLevels + 1];
    int n[kMaxLevels];
    int N[kMaxLevels];
    int cstride[kMaxLevels];
    const T* coef[kMaxLevels];
    int cst[kMaxLevels];       // constant stencil (coef holds 3^d values)
    const T* g[kMaxLevels];
    const T* c1[kMaxLevels];   // first sweep omega (g / D), written by the restriction
    const T* cin[kMaxLevels];
    T* cout[kMaxLevels];
};

// Damped Jacobi at one coarse node: first min(nu,2) sweeps (mode 0, c1 =
// omega g / D precomputed by the restriction) or one further sweep (mode 1).
template <int DIM, typename T>
__device__ __forceinline__ T coarse_smooth_at(const CoarseOp<T>& op, const T* __restrict__ g,
                                              const T* __restrict__ c1, const T* __restrict__ cin, int idx,
                                              T omega, int mode, int two_sweeps) {
    const Idx<DIM> p = decomp<DIM>(idx, op.n);
    const T gi = g[idx];
    const T Di = op.cst ? op.coef[stencil_center<DIM>()] : op.coef[(size_t)stencil_center<DIM>() * op.N + idx];
    if (mode == 0) {
        if (!two_sweeps) return c1[idx];
        const T Ac = coarse_apply_fn<DIM, T>(op, idx, p, [&](int j) -> T { return c1[j]; });
        return c1[idx] + omega * ((gi - Ac) / Di);
    }
    const T Ac = coarse_apply_fn<DIM, T>(op, idx, p, [&](int j) -> T { return cin[j]; });
    return cin[idx] + omega * ((gi - Ac) / Di);
}

// Block b of a level-fused coarse pass (blocks past blk_off[nlev] idle).
template <int DIM, typename T>
__device__ __forceinline__ void coarse_levels_block(const CoarseLevels<T>& L, int b, T omega, int mode,
                                                    int two_sweeps) {
    int l = 0;
    while (l + 1 < L.nlev && b >= L.blk_off[l + 1]) ++l;
    const int idx = (b - L.blk_off[l]) * kBlock + threadIdx.x;
    const int N = L.N[l];
    if (idx >= N) return;
    CoarseOp<T> op{L.n[l], N, L.coef[l], L.cst[l]};
    L.cout[l][(size_t)idx * L.cstride[l]] =
        coarse_smooth_at<DIM, T>(op, L.g[l], L.c1[l], L.cin[l], idx, omega, mode, two_sweeps);
}

template <int DIM, typename T>
__global__ void __launch_bounds__(kBlock) k_coarse_smooth(const Ctl* __restrict__ ctl, CoarseLevels<T> L,
                                                          T omega, int mode, int two_sweeps) {
    if (ctl->state != 0) return;
    coarse_levels_block<DIM, T>(L, (int)blockIdx.x, omega, mode, two_sweeps);
}

// One sweep index of every level in one launch (nu > 2): blocks [0, nbc)
// the level-fused coarse pass, the blocks after them the same pass on the
// finest level (mode 0: the first min(nu, 2) sweeps from r into fout;
// mode 1: one further sweep fin -> fout), over the row walk of grid - nbc
// blocks (nbc a multiple of 8 keeps the rows' XCD bands).  The levels are
// independent, so the sweeps of one index need no order among them.
template <int DIM, typename T>
__global__ void __launch_bounds__(kBlock) k_sweep_levels(const Ctl* __restrict__ ctl, CoarseLevels<T> L, int nbc,
                                                         T omega, int mode, int two, Rows R, FineOp<T> op,
                                                         const double* __restrict__ r, const T* __restrict__ fin,
                                                         T* __restrict__ fout) {
    if (ctl->state != 0) return;
    if ((int)blockIdx.x < nbc) {
        coarse_levels_block<DIM, T>(L, (int)blockIdx.x, omega, mode, two);
        return;
    }
    const Band b = row_band_of(R.total, (int)blockIdx.x - nbc, (int)gridDim.x - nbc);
    for (int w = b.start; w < b.end; w += b.stride) {
        Idx<DIM> p;
        int idx;
        if (!row_item<DIM>(R, w, p, idx)) continue;
        if (mode == 0) {
            fout[idx] = fine_smooth_at<DIM, T, double>(op, r, idx, p, omega, two);
        } else {
            const T res = T(r[idx]) - fine_apply<DIM, T>(op, fin, idx, p);
            fout[idx] = fin[idx] + omega * (res * fine_invdiag<DIM>(op, idx));
        }
    }
}

// Block carry up one level: Y_{l+1}[:, 0..NC-1] = P Y_l[:, 0..NC-1], both
// node-major (strides even_up(NC) and even_up(NC+1)).
template <int DIM, typename T, int NC>
__device__ __forceinline__ void prolong_at(const T* __restrict__ Yc, int nc, T* __restrict__ Yf, int nf, int idx) {
    constexpr int SC = even_up(NC), SF = even_up(NC + 1);
    const Idx<DIM> p = decomp<DIM>(idx, nf);
    const XPar px = xparents(p.i, nc);
    const Par py = parents(p.j, nc);
    const Par pz = DIM == 3 ? parents(p.k, nc) : Par{0, 0, 1.f, 0.f, 1};
    T z[SC];
    interp_block<DIM, T, SC>(Yc, nc, px, py, pz, z);
    T* o = Yf + (size_t)idx * SF;
#pragma unroll
    for (int c = 0; c < NC; ++c) o[c] = z[c];
}

// Block carry two levels up in one launch (level l -> l+2, NC = l + 1
// columns in Y_l): Y_{l+2}[:, 0..NC] = P [P Y_l | c_{l+1}] without storing
// level l+1's carried columns.  Each parent row of level l+1 is formed where
// it is needed exactly as the one-level carry stores it (the same
// interpolation from level l, then its own smoothed value c_{l+1}, already
// in Y_{l+1}, and the zero padding), so the results are those of two
// one-level launches.
template <int DIM, typename T, int NC>
__global__ void __launch_bounds__(kBlock) k_prolong2(const Ctl* __restrict__ ctl, const T* __restrict__ Yc, int nc,
                                                     const T* __restrict__ Ym, int nm, T* __restrict__ Yf, int nf,
                                                     int Nf) {
    if (ctl->state != 0) return;
    const int idx = blockIdx.x * kBlock + threadIdx.x;
    if (idx >= Nf) return;
    constexpr int SC = even_up(NC), SM = even_up(NC + 1), SF = even_up(NC + 2);
    const Idx<DIM> p = decomp<DIM>(idx, nf);
    const XPar px = xparents(p.i, nm);
    const Par py = parents(p.j, nm);
    const Par pz = DIM == 3 ? parents(p.k, nm) : Par{0, 0, 1.f, 0.f, 1};
    auto mid = [&](int I, int J, int K, T (&row)[SM]) {
        const XPar qx = xparents(I, nc);
        const Par qy = parents(J, nc);
        const Par qz = DIM == 3 ? parents(K, nc) : Par{0, 0, 1.f, 0.f, 1};
        T zc[SC];
        interp_block<DIM, T, SC>(Yc, nc, qx, qy, qz, zc);
        const T cm = Ym[((size_t)nm * (J + (size_t)nm * K) + I) * SM + NC];
#pragma unroll
        for (int c = 0; c < SM; ++c) row[c] = c < NC ? zc[c < SC ? c : 0] : (c == NC ? cm : T(0));
    };
    T z[SM];
    interp_block_fn<DIM, T, SM>(mid, px, py, pz, z);
    T* o = Yf + (size_t)idx * SF;
#pragma unroll
    for (int c = 0; c <= NC; ++c) o[c] = z[c];
}

template <int DIM, typename T, int NC>
__global__ void __launch_bounds__(kBlock) k_prolong(const Ctl* __restrict__ ctl, const T* __restrict__ Yc, int nc,
                                                    T* __restrict__ Yf, int nf, int Nf) {
    if (ctl->state != 0) return;
    const int idx = blockIdx.x * kBlock + threadIdx.x;
    if (idx >= Nf) return;
    prolong_at<DIM, T, NC>(Yc, nc, Yf, nf, idx);
}

// The small levels of the prolongation chain (levels l0 .. l0+count-1 to the
// next finer one) in one block, one level after the other.
template <typename T>
struct ProlongChain {
    int count, l0;
    int nc[kMaxLevels], nf[kMaxLevels], Nf[kMaxLevels];
    const T* Yc[kMaxLevels];
    T* Yf[kMaxLevels];
};

// The chain of ch.count prolongations, one level after the other, by one
// block of kTailBlock threads (all of them must call it).
template <int DIM, typename T>
__device__ __forceinline__ void prolong_chain_block(const ProlongChain<T>& ch) {
    for (int m = 0; m < ch.count; ++m) {
        const int NC = ch.l0 + m + 1;
        for (int idx = threadIdx.x; idx < ch.Nf[m]; idx += kTailBlock) {
            switch (NC) {
                case 1: prolong_at<DIM, T, 1>(ch.Yc[m], ch.nc[m], ch.Yf[m], ch.nf[m], idx); break;
                case 2: prolong_at<DIM, T, 2>(ch.Yc[m], ch.nc[m], ch.Yf[m], ch.nf[m], idx); break;
                case 3: prolong_at<DIM, T, 3>(ch.Yc[m], ch.nc[m], ch.Yf[m], ch.nf[m], idx); break;
                case 4: prolong_at<DIM, T, 4>(ch.Yc[m], ch.nc[m], ch.Yf[m], ch.nf[m], idx); break;
                case 5: prolong_at<DIM, T, 5>(ch.Yc[m], ch.nc[m], ch.Yf[m], ch.nf[m], idx); break;
                case 6: prolong_at<DIM, T, 6>(ch.Yc[m], ch.nc[m], ch.Yf[m], ch.nf[m], idx); break;
                default: prolong_at<DIM, T, 7>(ch.Yc[m], ch.nc[m], ch.Yf[m], ch.nf[m], idx); break;
            }
        }
        __syncthreads();
    }
}

template <int DIM, typename T>
__global__ void __launch_bounds__(kTailBlock) k_prolong_head(const Ctl* __restrict__ ctl, ProlongChain<T> ch) {
    if (ctl->state != 0) return;
    prolong_chain_block<DIM, T>(ch);
}

// --------------------------------------------- fused launches of the chain
//
// With nu <= 2 the additive levels leave much of the restriction/smoothing
// chain independent: the finest smoother and the first restriction read only
// r, and the smoother of level m+1 reads only what the restriction into
// m+1 wrote, as does the restriction m+1 -> m.  Each launch below runs one
// restriction in its first nbr blocks and one such smoother pass in the
// blocks after them, so their latencies overlap and the separate smoothing
// launches disappear.  The arithmetic is that of k_restrict, k_fine_smooth
// and k_coarse_smooth.

template <typename TI, typename T>
struct RestrictStep {
    const TI* gf;
    int nf;
    T* gc;
    int nc, Nc;
    const T* D;
    T* c1;
    int dconst;
};

// The first min(nu, 2) sweeps of one coarse level from zero, into out[i * stride].
template <typename T>
struct SmoothLevel {
    CoarseOp<T> op;
    const T* g;
    const T* c1;
    T* out;
    int stride;
};

template <int DIM, typename TI, typename T>
__device__ __forceinline__ void restrict_step(const RestrictStep<TI, T>& rs, int idx, T omega) {
    const T g = restrict_at<DIM, TI, T>(rs.gf, rs.nf, rs.nc, idx);
    rs.gc[idx] = g;
    rs.c1[idx] = omega * (g / rs.D[rs.dconst ? 0 : idx]);
}

template <int DIM, typename T>
__device__ __forceinline__ void smooth_level_at(const SmoothLevel<T>& sm, int idx, T omega, int two) {
    sm.out[(size_t)idx * sm.stride] = coarse_smooth_at<DIM, T>(sm.op, sm.g, sm.c1, nullptr, idx, omega, 0, two);
}

// Blocks [0, nbr): restriction r -> level L-1.  Blocks [nbr, grid): the
// finest smoother over the row walk of grid - nbr blocks (nbr is a multiple
// of 8, so the rows keep their XCD bands).
template <int DIM, typename T>
__global__ void __launch_bounds__(kBlock) k_restrict_fine_smooth(const Ctl* __restrict__ ctl,
                                                                 RestrictStep<double, T> rs, int nbr, Rows R,
                                                                 FineOp<T> op, const double* __restrict__ r,
                                                                 T* __restrict__ c, T omega, int two) {
    if (ctl->state != 0) return;
    if ((int)blockIdx.x < nbr) {
        // nbr is a multiple of 8: XCD x restricts the x-th band of coarse
        // nodes, which lies over the band of fine rows its smoother blocks read
        const int idx = xcd_block_of((int)blockIdx.x, nbr) * kBlock + threadIdx.x;
        if (idx < rs.Nc) restrict_step<DIM>(rs, idx, omega);
        return;
    }
    const Band b = row_band_of(R.total, (int)blockIdx.x - nbr, (int)gridDim.x - nbr);
    for (int w = b.start; w < b.end; w += b.stride) {
        Idx<DIM> p;
        int idx;
        if (!row_item<DIM>(R, w, p, idx)) continue;
        c[idx] = fine_smooth_at<DIM, T, double>(op, r, idx, p, omega, two);
    }
}

// 3D, constant coefficients, two sweeps: the restriction r -> level L-1 and
// the finest smoother from one LDS tile of r per block.  A block owns a
// kRTX x kRTY x kRTZ box of fine nodes (even corner), stages r over the box
// and a one-node halo (as T, zero outside the grid), smooths the box's nodes
// (4 per thread) and restricts the coarse nodes whose centre 2J+1 lies in the
// box (their 3^3 support lies in the staged halo).  The arithmetic, in its
// order, is that of fine_smooth_face without coefficient arrays and of
// restrict_at (a face neighbour outside the grid is weighted 0 and reads the
// halo's 0 instead of a clamped node), so the results are the same.  Tiles go
// to XCDs in contiguous runs (xcd_block_of): neighbouring boxes share a L2.
constexpr int kRTX = 32, kRTY = 8, kRTZ = 4;

template <typename T>
__global__ void __launch_bounds__(kBlock) k_restrict_fine_smooth_tile(const Ctl* __restrict__ ctl,
                                                                      RestrictStep<double, T> rs, FineOp<T> op,
                                                                      const double* __restrict__ r,
                                                                      T* __restrict__ c, T omega, int ntx, int nty,
                                                                      int ntz) {
    if (ctl->state != 0) return;
    static_assert(kRTX * kRTY == kBlock, "one thread per (x, y) of the box");
    constexpr int LX = kRTX + 2, LY = kRTY + 2, LZ = kRTZ + 2, NV = LX * LY * LZ;
    constexpr int NIT = (NV + kBlock - 1) / kBlock;
    __shared__ T tile[NV];
    const int t = xcd_block_of((int)blockIdx.x, ntx * nty * ntz);
    const int bx = t % ntx, by = (t / ntx) % nty, bz = t / (ntx * nty);
    const int X0 = bx * kRTX, Y0 = by * kRTY, Z0 = bz * kRTZ;
    const int n = op.n;
    // stage r over the box and its halo: all loads first
    T v[NIT];
#pragma unroll
    for (int q = 0; q < NIT; ++q) {
        const int vi = (int)threadIdx.x + q * kBlock;
        const int lx = vi % LX, ly = (vi / LX) % LY, lz = vi / (LX * LY);
        const int gx = X0 - 1 + lx, gy = Y0 - 1 + ly, gz = Z0 - 1 + lz;
        const bool in = vi < NV && gx >= 0 && gx < n && gy >= 0 && gy < n && gz >= 0 && gz < n;
        v[q] = in ? T(r[gx + n * (gy + n * gz)]) : T(0);
    }
#pragma unroll
    for (int q = 0; q < NIT; ++q) {
        const int vi = (int)threadIdx.x + q * kBlock;
        if (vi < NV) tile[vi] = v[q];
    }
    __syncthreads();
    // the finest smoother: c2 = c1 + omega ((g - A c1) / D), c1 = omega g / D
    const int sx = (int)threadIdx.x % kRTX, sy = (int)threadIdx.x / kRTX;
    const int x = X0 + sx, y = Y0 + sy;
#pragma unroll
    for (int k = 0; k < kRTZ; ++k) {
        const int z = Z0 + k;
        if (x >= n || y >= n || z >= n) continue;
        const T* tp = tile + ((k + 1) * LY + sy + 1) * LX + sx + 1;
        const T gi = tp[0];
        const T gq[6] = {tp[-1], tp[1], tp[-LX], tp[LX], tp[-LX * LY], tp[LX * LY]};
        const bool ok[6] = {x > 0, x < n - 1, y > 0, y < n - 1, z > 0, z < n - 1};
        const T c1 = omega * (gi * op.inv0);
        T acc = T(6) * c1;
#pragma unroll
        for (int q = 0; q < 6; ++q) acc -= (ok[q] ? T(1) : T(0)) * (omega * (gq[q] * op.inv0));
        const T Ac = op.s0 * acc;
        c[x + n * (y + n * z)] = c1 + omega * ((gi - Ac) * op.inv0);
    }
    // full weighting into level L-1 at the box's coarse nodes
    const int nf = rs.nf, nc = rs.nc;
    constexpr int CX = kRTX / 2, CY = kRTY / 2, CZ = kRTZ / 2;
    for (int j = threadIdx.x; j < CX * CY * CZ; j += kBlock) {
        const int Jx = X0 / 2 + j % CX, Jy = Y0 / 2 + (j / CX) % CY, Jz = Z0 / 2 + j / (CX * CY);
        if (Jx >= nc || Jy >= nc || Jz >= nc) continue;
        const int fx = 2 * Jx, fy = 2 * Jy, fz = 2 * Jz;
        const T w2x = fx + 2 < nf ? T(0.5) : T(0), w2y = fy + 2 < nf ? T(0.5) : T(0);
        const T w2z = fz + 2 < nf ? T(0.5) : T(0);
        // tile coordinates of the fine nodes 2J, 2J+1 and min(2J+2, nf-1)
        const int lx0 = fx - X0 + 1, lx2 = min(fx + 2, nf - 1) - X0 + 1;
        const int ly[3] = {fy - Y0 + 1, fy - Y0 + 2, min(fy + 2, nf - 1) - Y0 + 1};
        const int lz[3] = {fz - Z0 + 1, fz - Z0 + 2, min(fz + 2, nf - 1) - Z0 + 1};
        const T wy[3] = {T(0.5), T(1), w2y};
        const T wz[3] = {T(0.5), T(1), w2z};
        T acc = T(0);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            T plane = T(0);
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const T* rowp = tile + (lz[a] * LY + ly[b]) * LX;
                const T row = T(0.5) * rowp[lx0] + rowp[lx0 + 1] + w2x * rowp[lx2];
                plane += wy[b] * row;
            }
            acc += wz[a] * plane;
        }
        const T g = T(0.125) * acc;
        const int idx = Jx + nc * (Jy + nc * Jz);
        rs.gc[idx] = g;
        rs.c1[idx] = omega * (g / rs.D[rs.dconst ? 0 : idx]);
    }
}

// Blocks [0, nbr): restriction level m+1 -> m (nbr = 0: none).  Blocks
// [nbr, grid): the smoother of level m+1, one thread per node.
template <int DIM, typename T>
__global__ void __launch_bounds__(kBlock) k_restrict_coarse_smooth(const Ctl* __restrict__ ctl,
                                                                   RestrictStep<T, T> rs, int nbr,
                                                                   SmoothLevel<T> sm, T omega, int two) {
    if (ctl->state != 0) return;
    if ((int)blockIdx.x < nbr) {
        const int idx = blockIdx.x * kBlock + threadIdx.x;
        if (idx < rs.Nc) restrict_step<DIM>(rs, idx, omega);
        return;
    }
    const int idx = ((int)blockIdx.x - nbr) * kBlock + threadIdx.x;
    if (idx < sm.op.N) smooth_level_at<DIM>(sm, idx, omega, two);
}

// 3D, constant coarse stencil, two sweeps: the restriction level m+1 -> m
// and the smoother of level m+1 from one LDS box of level m+1's g and c1
// per block (kCBX x kCBY x kCBZ nodes, even corner, one-node halo, zero
// outside the grid).  The smoother's arithmetic and order are those of
// coarse_smooth_at (mode 0) and the restriction's those of restrict_at; a
// stencil tap outside the grid is weighted 0 and reads the halo's 0 instead
// of the node's own value, so the results are the same.
constexpr int kCBX = 16, kCBY = 4, kCBZ = 4;

template <typename T>
__global__ void __launch_bounds__(kBlock) k_restrict_coarse_smooth_tile(const Ctl* __restrict__ ctl,
                                                                        RestrictStep<T, T> rs, SmoothLevel<T> sm,
                                                                        T omega, int ntx, int nty, int ntz) {
    if (ctl->state != 0) return;
    static_assert(kCBX * kCBY * kCBZ == kBlock, "one thread per node of the box");
    constexpr int LX = kCBX + 2, LY = kCBY + 2, LZ = kCBZ + 2, NV = LX * LY * LZ;
    constexpr int NIT = (NV + kBlock - 1) / kBlock;
    __shared__ T tg[NV], tc[NV];
    const int t = xcd_block_of((int)blockIdx.x, ntx * nty * ntz);
    const int X0 = (t % ntx) * kCBX, Y0 = ((t / ntx) % nty) * kCBY, Z0 = (t / (ntx * nty)) * kCBZ;
    const int n = sm.op.n;
    T vg[NIT], vc[NIT];
#pragma unroll
    for (int q = 0; q < NIT; ++q) {
        const int vi = (int)threadIdx.x + q * kBlock;
        const int lx = vi % LX, ly = (vi / LX) % LY, lz = vi / (LX * LY);
        const int gx = X0 - 1 + lx, gy = Y0 - 1 + ly, gz = Z0 - 1 + lz;
        const bool in = vi < NV && gx >= 0 && gx < n && gy >= 0 && gy < n && gz >= 0 && gz < n;
        const int gi = in ? gx + n * (gy + n * gz) : 0;
        vg[q] = in ? sm.g[gi] : T(0);
        vc[q] = in ? sm.c1[gi] : T(0);
    }
#pragma unroll
    for (int q = 0; q < NIT; ++q) {
        const int vi = (int)threadIdx.x + q * kBlock;
        if (vi < NV) {
            tg[vi] = vg[q];
            tc[vi] = vc[q];
        }
    }
    __syncthreads();
    // the smoother of level m+1 at this thread's node
    {
        const int sx = (int)threadIdx.x % kCBX, sy = ((int)threadIdx.x / kCBX) % kCBY, sz = (int)threadIdx.x / (kCBX * kCBY);
        const int x = X0 + sx, y = Y0 + sy, z = Z0 + sz;
        if (x < n && y < n && z < n) {
            const int c0 = ((sz + 1) * LY + sy + 1) * LX + sx + 1;
            const T* __restrict__ coef = sm.op.coef;
            const T gi = tg[c0];
            const T Di = coef[stencil_center<3>()];
            T Ac = T(0);
            int s = 0;
#pragma unroll
            for (int dz = -1; dz <= 1; ++dz) {
                const bool okz = z + dz >= 0 && z + dz < n;
#pragma unroll
                for (int dy = -1; dy <= 1; ++dy) {
                    const bool oky = okz && y + dy >= 0 && y + dy < n;
#pragma unroll
                    for (int dx = -1; dx <= 1; ++dx, ++s) {
                        const bool ok = oky && x + dx >= 0 && x + dx < n;
                        const T w = coef[s];
                        Ac += (ok ? w : T(0)) * tc[c0 + dx + LX * (dy + LY * dz)];
                    }
                }
            }
            sm.out[(size_t)(x + n * (y + n * z)) * sm.stride] = tc[c0] + omega * ((gi - Ac) / Di);
        }
    }
    // the restriction into level m at the coarse nodes centred in the box
    const int nf = rs.nf, nc = rs.nc;
    constexpr int CX = kCBX / 2, CY = kCBY / 2, CZ = kCBZ / 2;
    for (int j = threadIdx.x; j < CX * CY * CZ; j += kBlock) {
        const int Jx = X0 / 2 + j % CX, Jy = Y0 / 2 + (j / CX) % CY, Jz = Z0 / 2 + j / (CX * CY);
        if (Jx >= nc || Jy >= nc || Jz >= nc) continue;
        const int fx = 2 * Jx, fy = 2 * Jy, fz = 2 * Jz;
        const T w2x = fx + 2 < nf ? T(0.5) : T(0), w2y = fy + 2 < nf ? T(0.5) : T(0);
        const T w2z = fz + 2 < nf ? T(0.5) : T(0);
        const int lx0 = fx - X0 + 1, lx2 = min(fx + 2, nf - 1) - X0 + 1;
        const int ly[3] = {fy - Y0 + 1, fy - Y0 + 2, min(fy + 2, nf - 1) - Y0 + 1};
        const int lz[3] = {fz - Z0 + 1, fz - Z0 + 2, min(fz + 2, nf - 1) - Z0 + 1};
        const T wy[3] = {T(0.5), T(1), w2y};
        const T wz[3] = {T(0.5), T(1), w2z};
        T acc = T(0);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            T plane = T(0);
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const T* rowp = tg + (lz[a] * LY + ly[b]) * LX;
                const T row = T(0.5) * rowp[lx0] + rowp[lx0 + 1] + w2x * rowp[lx2];
                plane += wy[b] * row;
            }
            acc += wz[a] * plane;
        }
        const T g = T(0.125) * acc;
        const int idx = Jx + nc * (Jy + nc * Jz);
        rs.gc[idx] = g;
        rs.c1[idx] = omega * (g / rs.D[rs.dconst ? 0 : idx]);
    }
}

// Block 0: the restriction chain into the small levels, one level after the
// other, the smoother of every small level, then the prolongation chain
// among them (up: coarsest first; it needs only what block 0 wrote).
// Blocks 1..: the smoother of the level the chain starts from.
template <typename T>
struct SmoothChain {
    int count;
    SmoothLevel<T> lev[kMaxLevels];
};

template <int DIM, typename T>
__global__ void __launch_bounds__(kTailBlock) k_tail_smooth(const Ctl* __restrict__ ctl, RestrictChain<T> ch,
                                                            SmoothChain<T> small, SmoothLevel<T> top,
                                                            ProlongChain<T> up, T omega, int two) {
    if (ctl->state != 0) return;
    if (blockIdx.x > 0) {
        const int idx = ((int)blockIdx.x - 1) * kTailBlock + threadIdx.x;
        if (idx < top.op.N) smooth_level_at<DIM>(top, idx, omega, two);
        return;
    }
    for (int m = 0; m < ch.count; ++m) {
        for (int idx = threadIdx.x; idx < ch.Nc[m]; idx += kTailBlock) {
            const T g = restrict_at<DIM, T, T>(ch.gf[m], ch.nf[m], ch.nc[m], idx);
            ch.gc[m][idx] = g;
            ch.c1[m][idx] = omega * (g / ch.D[m][ch.dconst[m] ? 0 : idx]);
        }
        __syncthreads();
    }
    // the small levels' smoothers side by side (each level its own range of
    // threads) when they fit in the block, else one level after the other
    int tot = 0;
    for (int q = 0; q < small.count; ++q) tot += small.lev[q].op.N;
    if (tot <= kTailBlock) {
        int off = 0;
        for (int q = 0; q < small.count; ++q) {
            const int idx = (int)threadIdx.x - off;
            if (idx >= 0 && idx < small.lev[q].op.N) smooth_level_at<DIM>(small.lev[q], idx, omega, two);
            off += small.lev[q].op.N;
        }
    } else {
        for (int q = 0; q < small.count; ++q)
            for (int idx = threadIdx.x; idx < small.lev[q].op.N; idx += kTailBlock)
                smooth_level_at<DIM>(small.lev[q], idx, omega, two);
    }
    if (up.count == 0) return;
    __syncthreads();
    prolong_chain_block<DIM, T>(up);
}

// Walk items per pass of the W kernel.
#ifndef AMG_W_ITEMS
#define AMG_W_ITEMS 1
#endif
constexpr int kWItems = AMG_W_ITEMS;

// W_j = Q_j^T Z_{k+1} partial sums (NB x NB, entry a*NB+c = Q_j column
// a . z^c) for the stored blocks j of the window in one launch: blocks
// [j nbs, (j+1) nbs) work on slot j (Q + j qstride, partials at
// part + j pstride), each range a full row walk of nbs blocks (nbs a
// multiple of 8 keeps every block on its XCD band).
template <int DIM, typename T, int NB, int NE>
__global__ void __launch_bounds__(kBlock) k_fine_W(const Ctl* __restrict__ ctl, Rows R, const T* __restrict__ Y,
                                                   int nc, const T* __restrict__ cL, const T* __restrict__ dl,
                                                   const int* __restrict__ dflag, const T* __restrict__ Q,
                                                   size_t qstride, double* __restrict__ part, size_t pstride,
                                                   int nbs) {
    if (ctl->state != 0) return;
    const bool dzero = NE && *dflag != 0;
    constexpr int S = even_up(NB);
    const int j = (int)blockIdx.x / nbs, bj = (int)blockIdx.x - j * nbs;
    Q += j * qstride;
    part += j * pstride;
    const int lb = xcd_block_of(bj, nbs);
    double w[NB * NB];
#pragma unroll
    for (int q = 0; q < NB * NB; ++q) w[q] = 0.0;
    const Band band = row_band_of(R.total, bj, nbs);
    // kWItems items of the walk per pass (items past the band end repeat the
    // first one and are not accumulated), every load of a pass issued before
    // any is used; the sums keep the walk's order
    constexpr int U = kWItems;
    for (int w_ = band.start; w_ < band.end; w_ += U * band.stride) {
        Idx<DIM> p[U];
        int idx[U], ix[U];
        bool act[U];
        ZWave<DIM, T, NB, NE> zw[U];
        T q[U][S];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int wu = w_ + u * band.stride < band.end ? w_ + u * band.stride : w_;   // uniform per wavefront
            act[u] = row_item<DIM>(R, wu, p[u], idx[u]) && (u == 0 || wu != w_);
            ix[u] = row_x(R, wu);
            fine_z_wave_load<DIM, T, NB, NE>(Y, nc, cL, dl, idx[u], p[u], ix[u], zw[u]);
            load_node<T, S>(Q + (size_t)idx[u] * S, q[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            T z[NB];
            fine_z_wave_finish<DIM, T, NB, NE>(zw[u], nc, dzero, p[u], ix[u], z);
            if (!act[u]) continue;
#pragma unroll
            for (int a = 0; a < NB; ++a) {
                const double qa = double(q[u][a]);
#pragma unroll
                for (int c = 0; c < NB; ++c) w[a * NB + c] += qa * double(z[c]);
            }
        }
    }
    block_sum_store<NB * NB>(w, part, nbs, lb);
}

// The stored direction blocks of the truncation window (a ring of m slots).
template <typename T>
struct PWin {
    T* p[kMaxWin];
};

// x += P_k alpha_k (deferred update of Algorithm 1); then, unless stopping,
// P_{k+1} = Z_{k+1} - sum_j P_j beta_j over the m stored blocks (slot cur
// holds P_k), written into slot nxt (the oldest, read first at each node);
// Z recomputed from the coarse block.  beta_j at beta + j kMaxNB^2.
// init = 1: P_0 = Z_0 only, into slot nxt.
// Blocks per CU the x/P update is compiled for.  Up to 6 columns, 5: the
// compiler then fits it into <= 94 VGPRs without spills, 5 waves per SIMD
// instead of 4 (measured: FP32 bulk 32.7 -> 29.7 us per launch at 127^3,
// FP64 the same), launched with one full round of resident blocks.  Wider
// blocks would spill at 5 and keep 4.
template <int NB>
__host__ __device__ constexpr int xp_blocks_per_cu() { return NB <= 6 ? 5 : 4; }

template <int DIM, typename T, int NB, int NE>
__global__ void __launch_bounds__(kBlock, (xp_blocks_per_cu<NB>())) k_update_xP(const Ctl* __restrict__ ctl, Rows R, const T* __restrict__ Y,
                                                      int nc, const T* __restrict__ cL, const T* __restrict__ dl,
                                                      const int* __restrict__ dflag, PWin<T> win, int m, int cur,
                                                      int nxt, double* __restrict__ x,
                                                      const double* __restrict__ alpha,
                                                      const double* __restrict__ beta, int init) {
    const int state = ctl->state;
    if (state == 2 || (init && state != 0)) return;
    const bool dzero = NE && *dflag != 0;
    constexpr int S = even_up(NB);
    const int lb = xcd_block(gridDim.x);
    __shared__ double sab[NB + kMaxWin * NB * NB];
    // per-wavefront staging of the FP64 block stores (FP32 nodes store
    // directly: measured faster at 24 bytes per node)
    constexpr bool kStage = sizeof(T) == 8;
    __shared__ __align__(16) T pbuf[kWaves][kStage ? 64 * S : 2];
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
    if (!init && state != 0) {
        // the stopping launch: the deferred x update alone
        ROW_LOOP(R, lb) {
            Idx<DIM> p;
            int idx;
            if (!row_item<DIM>(R, w_, p, idx)) continue;
            T pk[S];
            load_node<T, S>(Pc + (size_t)idx * S, pk);
            double xi = x[idx];
#pragma unroll
            for (int c = 0; c < NB; ++c) xi += double(pk[c]) * sab[c];
            x[idx] = xi;
        }
        return;
    }
    ROW_LOOP(R, lb) {
        Idx<DIM> p;
        int idx;
        const bool act = row_item<DIM>(R, w_, p, idx);
        const int ix = row_x(R, w_);
        // every load of the item first (P_k and x unless init, the coarse
        // parents, cL), then the arithmetic
        T pk[S];
        double xi = 0.0;
        if (!init) {
            load_node<T, S>(Pc + (size_t)idx * S, pk);
            xi = x[idx];
        }
        ZWave<DIM, T, NB, NE> zw;
        fine_z_wave_load<DIM, T, NB, NE>(Y, nc, cL, dl, idx, p, ix, zw);
        T z[NB];
        fine_z_wave_finish<DIM, T, NB, NE>(zw, nc, dzero, p, ix, z);
        // every lane computes (lanes past the row end on a clamped node) and,
        // in FP64, takes part in the wavefront's store of the new block
        double v[NB];
#pragma unroll
        for (int c = 0; c < NB; ++c) v[c] = double(z[c]);
        if (!init) {
#pragma unroll
            for (int c = 0; c < NB; ++c) xi += double(pk[c]) * sab[c];
            if (act) x[idx] = xi;
            const double* bc = sab + NB + cur * NB * NB;
#pragma unroll
            for (int c = 0; c < NB; ++c)
#pragma unroll
                for (int a2 = 0; a2 < NB; ++a2) v[c] -= double(pk[a2]) * bc[a2 * NB + c];
            for (int j = 0; j < m; ++j) {
                if (j == cur) continue;
                T pj[S];
                load_node<T, S>(win.p[j] + (size_t)idx * S, pj);
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
        if constexpr (kStage) {
            // lane 0 is always inside the row (row starts are multiples of
            // 64 below n), so its node starts the wavefront's range
            const int i0 = __builtin_amdgcn_readfirstlane(ix);
            const int first = __builtin_amdgcn_readfirstlane(idx);
            store_nodes_wave<T, S>(Pn + (size_t)first * S, min(64, R.n - i0), pbuf[threadIdx.x >> 6], pn);
        } else if (act) {
            store_node<T, S>(Pn + (size_t)idx * S, pn);
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
    constexpr int S = even_up(NB);
    const int lb = xcd_block(gridDim.x);
    double acc[NG + NB];
#pragma unroll
    for (int q = 0; q < NG + NB; ++q) acc[q] = 0.0;
    ROW_LOOP(R, lb) {
        Idx<DIM> p;
        int idx;
        if (!row_item<DIM>(R, w_, p, idx)) continue;
        T pv[S], qv[S];
        fine_apply_block<DIM, T, S>(op, P, idx, p, pv, qv);
        store_node<T, S>(Q + (size_t)idx * S, qv);
        const double ri = r[idx];
        int q = 0;
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int c = a; c < NB; ++c) acc[q++] += double(pv[a]) * double(qv[c]);
#pragma unroll
        for (int a = 0; a < NB; ++a) acc[NG + a] += double(pv[a]) * ri;
    }
    block_sum_store<NG + NB>(acc, part, gridDim.x, lb);
}

// ------------------------------------------- z-marching block SpMM (3D)
//
// The same Q = A P and Gram partials as k_spmm_gram, for 3D grids, with the
// work split into units of (an x tile of kZTileX nodes) x (TY rows) x (kz
// planes).  A block marches its unit along z.  The plane it works on and the
// next one sit in LDS with a one-node halo in x and a one-row halo in y; the
// block fills them with 16-byte chunk loads that read every row segment
// contiguously (the node-major block is one run of bytes per row), and keeps
// each node's value one plane down in registers.  P is thus read from global
// memory about once per unit, plus the halos, with full-width loads, instead
// of as seven strided node loads per node.
constexpr int kZTileX = 128;

template <typename T, int NB>
struct ZTile {
    static constexpr int S = even_up(NB);
    static constexpr int NODE = S * (int)sizeof(T);            // bytes per node
    static constexpr int U = NODE % 16 == 0 ? 1 : 2;           // nodes per 16-byte step
    // nodes i0-1 .. i0+kZTileX, from a U-aligned start, rounded to U nodes
    static constexpr int L = (kZTileX + 2 + (U - 1) + U - 1) / U * U;
    static constexpr int CR = L * NODE / 16;                   // chunks per row segment
};

// Flat index of the first node of the segment of row (j, k) of the tile
// starting at x = i0, and that node's offset (0 .. U-1) below the wanted
// first node i0 - 1.
template <int U>
__device__ __forceinline__ long long zt_start(int n, int i0, int j, int k, int& off) {
    const long long f = ((long long)k * n + j) * n + i0 - 1;
    const int m = U == 1 ? 0 : (int)(((f % U) + U) % U);
    off = m;
    return f - m;
}

// Chunks of plane k (rows j0-1 .. j0+TY) into registers; chunks outside
// [0, pbytes) and rows or planes outside the grid are left as zeros.
template <typename T, int NB, int TY, int CPT>
__device__ __forceinline__ void zt_fetch(const char* __restrict__ P, long long pbytes, int n, int i0, int j0, int k,
                                         uint4 (&buf)[CPT]) {
    using Z = ZTile<T, NB>;
    constexpr int C = (TY + 2) * Z::CR;
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        buf[q] = make_uint4(0u, 0u, 0u, 0u);
        const int c = (int)threadIdx.x + q * kBlock;
        if (c >= C || k < 0 || k >= n) continue;
        const int row = c / Z::CR, cc = c - row * Z::CR;
        const int j = j0 - 1 + row;
        if (j < 0 || j >= n) continue;
        int off;
        const long long b = zt_start<Z::U>(n, i0, j, k, off) * Z::NODE + (long long)cc * 16;
        if (b >= 0 && b + 16 <= pbytes) buf[q] = *reinterpret_cast<const uint4*>(P + b);
    }
}

template <typename T, int NB, int TY, int CPT>
__device__ __forceinline__ void zt_put(char* slot, const uint4 (&buf)[CPT]) {
    using Z = ZTile<T, NB>;
    constexpr int C = (TY + 2) * Z::CR;
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        const int c = (int)threadIdx.x + q * kBlock;
        if (c < C) reinterpret_cast<uint4*>(slot)[c] = buf[q];
    }
}

// Node (x, y) of the tile (x in -1 .. kZTileX, y in -1 .. TY) in a slot
// holding plane k.
template <typename T, int NB>
__device__ __forceinline__ const T* zt_node(const char* slot, int n, int i0, int j0, int k, int x, int y) {
    using Z = ZTile<T, NB>;
    int off = 0;
    if (Z::U > 1) (void)zt_start<Z::U>(n, i0, j0 + y, k, off);
    return reinterpret_cast<const T*>(slot + ((y + 1) * Z::L + x + 1 + off) * Z::NODE);
}

// Per-node operands of one plane step: r and the variable coefficients.
template <typename T>
struct ZOps {
    double r;
    T d, exm, exp, eym, eyp, ezp;
};

// The z-marching SpMM serves blocks of at most 48 bytes per node (FP64 up to
// six columns, FP32 up to eight) and seven FP64 columns (64 bytes, two
// blocks per CU); eight FP64 columns would spill and take the row-mapped
// kernel.
template <typename T, int NB>
__host__ __device__ constexpr bool zt_fits() { return even_up(NB) * (int)sizeof(T) <= 48 || NB == 7; }

template <typename T, int NPT, int RPP, bool VAR>
__device__ __forceinline__ void zt_ops(const FineOp<T>& op, const double* __restrict__ r, int n, int i, int j0, int yl,
                                       int k, ZOps<T> (&o)[NPT]) {
    const long long sy = n;
#pragma unroll
    for (int s = 0; s < NPT; ++s) {
        const int j = j0 + yl + RPP * s;
        o[s].r = 0.0;
        o[s].d = o[s].exm = o[s].exp = o[s].eym = o[s].eyp = o[s].ezp = T(0);
        if (i < n && j < n) {
            const long long idx = ((long long)k * n + j) * n + i;
            o[s].r = r[idx];
            if (VAR) {
                o[s].d = op.D[idx];
                if (i > 0) o[s].exm = op.ex[idx - 1];
                if (i < n - 1) o[s].exp = op.ex[idx];
                if (j > 0) o[s].eym = op.ey[idx - sy];
                if (j < n - 1) o[s].eyp = op.ey[idx];
                if (k < n - 1) o[s].ezp = op.ez[idx];
            }
        }
    }
}

// One unit per block: lb = (ty * nkz + kc) * ntx + tx (XCD-contiguous ranges
// of lb are slabs of y tiles with all their z chunks).  pbytes: readable
// bytes from P.  Each thread owns x = t mod kZTileX and rows
// y = t / kZTileX + 2 s.  Each step first issues the loads of the next
// step's per-node operands and the chunks of the plane after next, then
// works on LDS and registers only, so the loads stay in flight across it.
// VAR: variable coefficients (op.D, ex, ey, ez), else the constant h^-2
// stencil.  Three blocks of 4 waves fit a CU (LDS of the FP64 six-column tile
// ~51 KB); the variable-coefficient kernels on wide blocks carry the next
// step's coefficients as well and get two, which keeps them free of spills,
// and so do tiles of 64-byte nodes (~67 KB of LDS).
template <typename T, int NB, bool VAR>
__host__ __device__ constexpr int zt_min_blocks() {
    return (even_up(NB) * (int)sizeof(T) > 48 || (VAR && (sizeof(T) == 8 ? NB >= 5 : NB >= 7))) ? 2 : 3;
}
template <typename T, int NB, int TY, bool VAR>
__global__ void __launch_bounds__(kBlock, (zt_min_blocks<T, NB, VAR>())) k_spmm_gram_z(const Ctl* __restrict__ ctl, int n, int ntx, int kz,
                                                           int nkz, FineOp<T> op, const T* __restrict__ P,
                                                           long long pbytes, T* __restrict__ Q,
                                                           const double* __restrict__ r, double* __restrict__ part) {
    if (ctl->state != 0) return;
    using Z = ZTile<T, NB>;
    constexpr int S = Z::S;
    constexpr int NG = NB * (NB + 1) / 2;
    constexpr int RPP = kBlock / kZTileX;                        // rows per pass
    static_assert(TY % RPP == 0, "TY must be a multiple of the rows per pass");
    constexpr int NPT = TY / RPP;                                // nodes per thread and plane
    constexpr int SLOT = (TY + 2) * Z::L * Z::NODE;
    constexpr int CPT = ((TY + 2) * Z::CR + kBlock - 1) / kBlock;
    __shared__ __align__(16) char lds[2 * SLOT];

    const int lb = xcd_block(gridDim.x);
    const int tx = lb % ntx, rest = lb / ntx;
    const int kc = rest % nkz, ty = rest / nkz;
    const int i0 = tx * kZTileX, j0 = ty * TY, k0 = kc * kz, k1 = min(n, k0 + kz);
    const int xl = (int)threadIdx.x % kZTileX, yl = (int)threadIdx.x / kZTileX;
    const int i = i0 + xl;
    const char* Pb = reinterpret_cast<const char*>(P);
    constexpr bool var = VAR;

    double acc[NG + NB];
#pragma unroll
    for (int q = 0; q < NG + NB; ++q) acc[q] = 0.0;
    T pm[NPT][S];     // own node, plane k - 1
    T ezm[NPT];       // ez between planes k - 1 and k (variable coefficient)
#pragma unroll
    for (int s = 0; s < NPT; ++s) {
        const int j = j0 + yl + RPP * s;
#pragma unroll
        for (int c = 0; c < S; ++c) pm[s][c] = T(0);
        ezm[s] = T(0);
        if (i < n && j < n && k0 > 0 && k0 < n) {
            const long long idx = ((long long)(k0 - 1) * n + j) * n + i;
            load_node<T, S>(P + idx * S, pm[s]);
            if (var) ezm[s] = op.ez[idx];
        }
    }
    const int klast = min(k1, n - 1);       // last plane a step reads
    ZOps<T> ops[NPT];
    zt_ops<T, NPT, RPP, VAR>(op, r, n, i, j0, yl, k0, ops);
    uint4 buf[CPT];
    zt_fetch<T, NB, TY, CPT>(Pb, pbytes, n, i0, j0, k0, buf);
    zt_put<T, NB, TY, CPT>(lds, buf);
    if (k0 + 1 <= klast) {
        zt_fetch<T, NB, TY, CPT>(Pb, pbytes, n, i0, j0, k0 + 1, buf);
        zt_put<T, NB, TY, CPT>(lds + SLOT, buf);
    }
    __syncthreads();
    int cur = 0;
    for (int k = k0; k < k1; ++k) {
        ZOps<T> nops[NPT];
        if (k + 1 < k1) zt_ops<T, NPT, RPP, VAR>(op, r, n, i, j0, yl, k + 1, nops);
        const bool more = k + 2 <= klast;
        if (more) zt_fetch<T, NB, TY, CPT>(Pb, pbytes, n, i0, j0, k + 2, buf);
        const char* sc = lds + cur * SLOT;
        const char* sn = lds + (cur ^ 1) * SLOT;
#pragma unroll
        for (int s = 0; s < NPT; ++s) {
            const int y = yl + RPP * s, j = j0 + y;
            if (i >= n || j >= n) continue;
            const long long idx = ((long long)k * n + j) * n + i;
            T own[S], q[S], nb[S];
            load_node<T, S>(zt_node<T, NB>(sc, n, i0, j0, k, xl, y), own);
            if constexpr (!var) {
#pragma unroll
                for (int c = 0; c < S; ++c) q[c] = T(6) * own[c];
                auto sub = [&](const T* src) {
                    load_node<T, S>(src, nb);
#pragma unroll
                    for (int c = 0; c < S; ++c) q[c] -= nb[c];
                };
                if (i > 0) sub(zt_node<T, NB>(sc, n, i0, j0, k, xl - 1, y));
                if (i < n - 1) sub(zt_node<T, NB>(sc, n, i0, j0, k, xl + 1, y));
                if (j > 0) sub(zt_node<T, NB>(sc, n, i0, j0, k, xl, y - 1));
                if (j < n - 1) sub(zt_node<T, NB>(sc, n, i0, j0, k, xl, y + 1));
                if (k > 0) {
#pragma unroll
                    for (int c = 0; c < S; ++c) q[c] -= pm[s][c];
                }
                if (k < n - 1) sub(zt_node<T, NB>(sn, n, i0, j0, k + 1, xl, y));
#pragma unroll
                for (int c = 0; c < S; ++c) q[c] *= op.s0;
            } else {
#pragma unroll
                for (int c = 0; c < S; ++c) q[c] = ops[s].d * own[c];
                auto sub = [&](const T* src, T e) {
                    load_node<T, S>(src, nb);
#pragma unroll
                    for (int c = 0; c < S; ++c) q[c] -= e * nb[c];
                };
                if (i > 0) sub(zt_node<T, NB>(sc, n, i0, j0, k, xl - 1, y), ops[s].exm);
                if (i < n - 1) sub(zt_node<T, NB>(sc, n, i0, j0, k, xl + 1, y), ops[s].exp);
                if (j > 0) sub(zt_node<T, NB>(sc, n, i0, j0, k, xl, y - 1), ops[s].eym);
                if (j < n - 1) sub(zt_node<T, NB>(sc, n, i0, j0, k, xl, y + 1), ops[s].eyp);
                if (k > 0) {
#pragma unroll
                    for (int c = 0; c < S; ++c) q[c] -= ezm[s] * pm[s][c];
                }
                if (k < n - 1) sub(zt_node<T, NB>(sn, n, i0, j0, k + 1, xl, y), ops[s].ezp);
                ezm[s] = ops[s].ezp;
            }
            store_node<T, S>(Q + idx * S, q);
            int g = 0;
#pragma unroll
            for (int a = 0; a < NB; ++a)
#pragma unroll
                for (int c = a; c < NB; ++c) acc[g++] += double(own[a]) * double(q[c]);
#pragma unroll
            for (int a = 0; a < NB; ++a) acc[NG + a] += double(own[a]) * ops[s].r;
#pragma unroll
            for (int c = 0; c < S; ++c) pm[s][c] = own[c];
        }
#pragma unroll
        for (int s = 0; s < NPT; ++s) ops[s] = nops[s];
        __syncthreads();
        if (more) zt_put<T, NB, TY, CPT>(lds + cur * SLOT, buf);
        __syncthreads();
        cur ^= 1;
    }
    block_sum_store<NG + NB>(acc, part, gridDim.x, lb);
}

// Explicit Z (widened to double, column-major), for the mg_block entry point.
template <int DIM, typename T, int NB, int NE>
__global__ void __launch_bounds__(kBlock) k_write_Z(Rows R, int N, const T* __restrict__ Y, int nc,
                                                    const T* __restrict__ cL, const T* __restrict__ dl,
                                                    const int* __restrict__ dflag, double* __restrict__ Z) {
    const bool dzero = NE && *dflag != 0;
    ROW_LOOP(R, blockIdx.x) {
        Idx<DIM> p;
        int idx;
        const bool act = row_item<DIM>(R, w_, p, idx);
        T z[NB];
        fine_z_wave<DIM, T, NB, NE>(Y, nc, cL, dl, dzero, idx, p, row_x(R, w_), z);
        if (!act) continue;
#pragma unroll
        for (int c = 0; c < NB; ++c) Z[(size_t)c * N + idx] = double(z[c]);
    }
}

// b == 0: x = 0.
static __global__ void __launch_bounds__(kBlock) k_zero_if(const Ctl* __restrict__ ctl, double* __restrict__ x, int N) {
    if (!ctl->zero_x) return;
    for (int idx = blockIdx.x * kBlock + threadIdx.x; idx < N; idx += gridDim.x * kBlock) x[idx] = 0.0;
}

}  // namespace amg
