// The comparison methods of Sec. 3 on the same hierarchy and kernels: CG
// with one search direction per iteration, preconditioned either by the sum
// of the additive level corrections (eq. (3)) or by one multiplicative
// V-cycle (Sec. 2.1: smoothing on the way from the finest to the coarsest
// level and back).  The outer loop is the MPCG machinery with one column --
// A-orthogonalisation p_{k+1} = z_{k+1} - p_k beta, beta = (q_k . z_{k+1}) /
// (p_k . q_k), which is the CG recurrence for a symmetric preconditioner --
// so the SpMM/Gram, residual update and the two single-block reductions are
// shared.  One-column blocks keep the node stride 2 (even_up(1)).
#pragma once

#include "grid_kernels.hpp"

namespace amg {

// z = sum of the NL level corrections at every fine node (the additive MG
// preconditioner of eq. (3)), formed from the level-(L-1) block carry and the
// finest smoother output exactly like the MPCG directions, added coarsest
// first.
template <int DIM, typename T, int NL>
__global__ void __launch_bounds__(kBlock) k_sum_z(const Ctl* __restrict__ ctl, Rows R, const T* __restrict__ Y,
                                                  int nc, const T* __restrict__ cL, T* __restrict__ z) {
    if (ctl->state != 0) return;
    ROW_LOOP(R, blockIdx.x) {
        Idx<DIM> p;
        int idx;
        const bool act = row_item<DIM>(R, w_, p, idx);
        T zc[NL];
        fine_z_wave<DIM, T, NL, 0>(Y, nc, cL, nullptr, false, idx, p, row_x(R, w_), zc);
        if (!act) continue;
        T s = zc[0];
#pragma unroll
        for (int c = 1; c < NL; ++c) s += zc[c];
        z[idx] = s;
    }
}

// W = q_k . z_{k+1} partial sums (one column, stride 2).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_W1(const Ctl* __restrict__ ctl, int N, const T* __restrict__ Q,
                                               const T* __restrict__ z, double* __restrict__ part) {
    if (ctl->state != 0) return;
    const int lb = xcd_block(gridDim.x);
    double v[1] = {0.0};
    const int per = ((N + gridDim.x - 1) / gridDim.x + kBlock - 1) / kBlock * kBlock;
    const int end = min(N, (lb + 1) * per);
    for (int idx = lb * per + threadIdx.x; idx < end; idx += kBlock)
        v[0] += double(Q[(size_t)idx * 2]) * double(z[idx]);
    block_sum_store<1>(v, part, gridDim.x, lb);
}

// x += alpha p_k (deferred update); then, unless stopping,
// p_{k+1} = z_{k+1} - beta p_k in place.  init = 1: p_0 = z_0 only.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_xP1(const Ctl* __restrict__ ctl, int N, T* __restrict__ P,
                                                const T* __restrict__ z, double* __restrict__ x,
                                                const double* __restrict__ alpha, const double* __restrict__ beta,
                                                int init) {
    const int state = ctl->state;
    if (state == 2 || (init && state != 0)) return;
    const double a = init ? 0.0 : alpha[0];
    const double bt = init ? 0.0 : beta[0];
    for (int idx = blockIdx.x * kBlock + threadIdx.x; idx < N; idx += gridDim.x * kBlock) {
        T* pp = P + (size_t)idx * 2;
        if (init) {
            pp[0] = z[idx];
            pp[1] = T(0);
            continue;
        }
        const double pk = double(pp[0]);
        x[idx] += pk * a;
        if (state != 0) continue;
        pp[0] = T(double(z[idx]) - pk * bt);
    }
}

// ------------------------------------------------------------- V-cycle

// Finest-level residual res = g - A c (type T).
template <int DIM, typename T, typename G>
__global__ void __launch_bounds__(kBlock) k_fine_resid(const Ctl* __restrict__ ctl, Rows R, FineOp<T> op,
                                                       const G* __restrict__ g, const T* __restrict__ c,
                                                       T* __restrict__ res) {
    if (ctl->state != 0) return;
    ROW_LOOP(R, blockIdx.x) {
        Idx<DIM> p;
        int idx;
        if (!row_item<DIM>(R, w_, p, idx)) continue;
        res[idx] = T(g[idx]) - fine_apply<DIM, T>(op, c, idx, p);
    }
}

// One coarse level of the V-cycle, thread per node.  mode 1: one damped
// Jacobi sweep cout = cin + omega ((g - A cin) / D) (eq. (2)); mode 2: the
// residual cout = g - A cin.
template <int DIM, typename T>
__global__ void __launch_bounds__(kBlock) k_vc_coarse(const Ctl* __restrict__ ctl, CoarseOp<T> op,
                                                      const T* __restrict__ g, const T* __restrict__ cin,
                                                      T* __restrict__ cout, T omega, int mode) {
    if (ctl->state != 0) return;
    const int idx = blockIdx.x * kBlock + threadIdx.x;
    if (idx >= op.N) return;
    const Idx<DIM> p = decomp<DIM>(idx, op.n);
    const T Ac = coarse_apply_fn<DIM, T>(op, idx, p, [&](int j) -> T { return cin[j]; });
    const T res = g[idx] - Ac;
    if (mode == 2) {
        cout[idx] = res;
        return;
    }
    const T Di = op.cst ? op.coef[stencil_center<DIM>()] : op.coef[(size_t)stencil_center<DIM>() * op.N + idx];
    cout[idx] = cin[idx] + omega * (res / Di);
}

// Coarse-grid correction c_f += P c_c (linear interpolation of one coarse
// vector, coarse node J on fine node 2J+1), thread per fine node.
template <int DIM, typename T>
__global__ void __launch_bounds__(kBlock) k_prolong_add(const Ctl* __restrict__ ctl, const T* __restrict__ cc,
                                                        int nc, T* __restrict__ cf, int nf, int Nf) {
    if (ctl->state != 0) return;
    const int idx = blockIdx.x * kBlock + threadIdx.x;
    if (idx >= Nf) return;
    const Idx<DIM> p = decomp<DIM>(idx, nf);
    cf[idx] += interp_at<DIM, T, T>(cc, nc, p);
}

}  // namespace amg
