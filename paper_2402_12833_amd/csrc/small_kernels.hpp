// Single-block kernels: the global reductions of one iteration, the b x b
// pseudo-inverse of the Gram matrix, the step coefficients alpha and beta,
// convergence and stop logic.  They run as one 1024-thread block; the
// eigen-decomposition runs in wavefront 0 with one Gram entry per lane.
#pragma once

#include "common.hpp"

namespace amg {

// Status codes mirrored from the public header (kept numerically equal).
constexpr int kOK = 0, kMAXIT = 1, kBREAKDOWN = 2, kNONFINITE = -4;

// In-place Gauss-Jordan inversion of a symmetric positive definite NB x NB
// matrix held one entry per lane (lane l < NB*NB owns (i, j)); no pivoting.
// ok becomes false if a pivot is not positive (then the content is garbage).
template <int NB>
__device__ __forceinline__ void wave_gauss_jordan(double& a, int i, int j, bool live, bool& ok) {
    for (int p = 0; p < NB; ++p) {
        const double piv = __shfl(a, p * NB + p);
        const double apj = __shfl(a, p * NB + j);
        const double aip = __shfl(a, i * NB + p);
        if (!(piv > 0.0)) {
            ok = false;
            return;
        }
        const double rpj = ((j == p) ? 1.0 : apj) / piv;
        const double a2 = (i == p) ? rpj : ((j == p) ? 0.0 : a) - aip * rpj;
        a = live ? a2 : 0.0;
    }
}

// Pseudo-inverse of a symmetric PSD NB x NB matrix G (row-major, shared
// memory) by cyclic Jacobi on the unit-diagonal scaling Ghat = S G S,
// S = diag(G_ii^{-1/2}) over the active columns (finite, positive diagonal).
// Eigenvalues <= tau are dropped; G^+ = S V Lambda^+ V^T S.  Must be called
// by all 64 lanes of one wavefront; lane l < NB*NB owns entry (l / NB, l % NB).
// Writes Gplus (row-major) and returns the rank to every lane.
template <int NB>
__device__ int wave_pinv(const double* G, double tau, double* Gplus) {
    const int lane = threadIdx.x & 63;
    const bool live = lane < NB * NB;
    const int i = live ? lane / NB : 0, j = live ? lane % NB : 0;
    const double gii = G[i * NB + i], gjj = G[j * NB + j], gij = G[i * NB + j];
    const bool ai = isfinite(gii) && gii > 0.0, aj = isfinite(gjj) && gjj > 0.0;
    const double si = ai ? 1.0 / sqrt(gii) : 0.0, sj = aj ? 1.0 / sqrt(gjj) : 0.0;
    const bool bad = live && ai && aj && !isfinite(gij);
    if (__any(bad)) {
        if (live) Gplus[lane] = 0.0;
        return 0;
    }
    double a = (live && ai && aj) ? (gij * si) * sj : 0.0;
    // Fast path: if Ghat - 2 tau I is positive definite (all Gauss-Jordan
    // pivots positive), no eigenvalue of Ghat is <= tau, so the pseudo-inverse
    // is the inverse; it is formed by in-place Gauss-Jordan.  Otherwise the
    // eigen-decomposition below applies the cut.
    {
        bool ok = true;
        double shifted = a - ((live && i == j) ? 2.0 * tau : 0.0);
        wave_gauss_jordan<NB>(shifted, i, j, live, ok);
        if (ok) {
            double inv = a;
            wave_gauss_jordan<NB>(inv, i, j, live, ok);
            if (ok) {
                if (live) Gplus[lane] = si * inv * sj;
                return NB;
            }
        }
    }
    double v = (live && i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 30; ++sweep) {
        const double off = wave_sum((live && i != j) ? a * a : 0.0);
        const double fro = wave_sum(live ? a * a : 0.0);
        if (!(off > 1e-30 * fro)) break;
        for (int p = 0; p < NB - 1; ++p) {
            for (int q = p + 1; q < NB; ++q) {
                const double apq = __shfl(a, p * NB + q);
                if (apq == 0.0) continue;
                const double app = __shfl(a, p * NB + p), aqq = __shfl(a, q * NB + q);
                // rotation zeroing (p,q): cot(2 theta) = (aqq - app) / (2 apq)
                const double zeta = (aqq - app) / (2.0 * apq);
                const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(zeta * zeta + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                // columns p, q of A J
                const double aip = __shfl(a, i * NB + p), aiq = __shfl(a, i * NB + q);
                double bb = a;
                if (j == p) bb = c * aip - s * aiq;
                else if (j == q) bb = s * aip + c * aiq;
                // rows p, q of J^T (A J)
                const double bpj = __shfl(bb, p * NB + j), bqj = __shfl(bb, q * NB + j);
                double a2 = bb;
                if (i == p) a2 = c * bpj - s * bqj;
                else if (i == q) a2 = s * bpj + c * bqj;
                if ((i == p && j == q) || (i == q && j == p)) a2 = 0.0;
                a = live ? a2 : 0.0;
                // V J
                const double vip = __shfl(v, i * NB + p), viq = __shfl(v, i * NB + q);
                if (j == p) v = c * vip - s * viq;
                else if (j == q) v = s * vip + c * viq;
            }
        }
    }
    double gp = 0.0;
    int rank = 0;
    for (int k = 0; k < NB; ++k) {
        const double lam = __shfl(a, k * NB + k);
        const double vik = __shfl(v, i * NB + k), vjk = __shfl(v, j * NB + k);
        if (lam > tau) {
            gp += vik * vjk / lam;
            ++rank;
        }
    }
    if (live) Gplus[lane] = si * gp * sj;
    return rank;
}

// After the init residual: ||b||, ||r_0||, stop if r_0 already small.
// One thread, given the sums ||b||^2 and ||r_0||^2.
__device__ __forceinline__ void init_decide(Ctl* ctl, double bn2, double rho, double tol, double* rhist) {
    ctl->bnorm2 = bn2;
    ctl->tol2 = tol * tol * bn2;
    ctl->rho = rho;
    ctl->rho_ref = rho;
    ctl->it = 0;
    ctl->refreshes = 0;
    ctl->refresh_req = 0;
    ctl->zero_x = 0;
    ctl->status = kOK;
    ctl->state = 0;
    if (rhist && ctl->hist_cap > 0) rhist[0] = sqrt(rho);
    if (bn2 == 0.0) {
        ctl->zero_x = 1;
        ctl->state = 2;
    } else if (!isfinite(rho) || !isfinite(bn2)) {
        ctl->status = kNONFINITE;
        ctl->state = 2;
    } else if (rho <= ctl->tol2) {
        ctl->state = 2;
    }
}

__device__ __forceinline__ void reduce_init_body(Ctl* ctl, const double* part, int nblk, double tol,
                                                 double* rhist) {
    __shared__ double res[2];
    reduce_partials<2>(part, nblk, res);
    if (threadIdx.x != 0) return;
    init_decide(ctl, res[0], res[1], tol, rhist);
}

static __global__ void __launch_bounds__(kRedBlock) k_reduce_init(Ctl* ctl, const double* part, int nblk, double tol,
                                                        double* rhist) {
    reduce_init_body(ctl, part, nblk, tol, rhist);
}

// The true relative residual ||b - A x|| / ||b|| of the returned iterate,
// from the partials (||b||^2, ||r||^2) of the FP64 residual kernel.
static __global__ void __launch_bounds__(kRedBlock) k_true_relres(Ctl* ctl, const double* part, int nblk) {
    __shared__ double res[2];
    reduce_partials<2>(part, nblk, res);
    if (threadIdx.x == 0) ctl->relres_true = res[0] > 0.0 ? sqrt(res[1] / res[0]) : 0.0;
}

// Residual check of r_{k+1} (one thread, given rho = ||r_{k+1}||^2): counts
// the x update, stops on convergence, a non-finite residual or maxit, and
// in the mixed form (mixed != 0) only requests a true-residual refresh on
// convergence of the recursive residual (the refresh decides).  Returns the
// new state (0 running, 1 stop after the pending x update).
__device__ __forceinline__ int beta_decide(Ctl* ctl, double rho, double* rhist, int mixed) {
    const int it = ctl->it + 1;
    ctl->it = it;
    ctl->rho = rho;
    if (rhist && it < ctl->hist_cap + 1) rhist[it] = sqrt(rho);
    int st = 0;
    if (!isfinite(rho)) {
        ctl->status = kNONFINITE;
        st = 1;
    } else if (rho <= ctl->tol2 && !mixed) {
        ctl->status = kOK;
        st = 1;
    } else if (it >= ctl->maxit) {
        ctl->status = kMAXIT;
        st = 1;
    } else if (mixed && (rho <= ctl->tol2 || rho <= ctl->drop2 * ctl->rho_ref)) {
        ctl->refresh_req = 1;
    }
    ctl->state = st;
    return st;
}

// beta = G^+ W (NB x NB), entries q = tid, tid + nt, ... of this thread.
template <int NB>
__device__ __forceinline__ void beta_apply(const double* Gplus, const double* W, double* beta, int tid, int nt) {
    for (int q = tid; q < NB * NB; q += nt) {
        const int a = q / NB, c = q % NB;
        double s = 0.0;
        for (int m = 0; m < NB; ++m) s += Gplus[a * NB + m] * W[m * NB + c];
        beta[q] = s;
    }
}

// Residual check of r_{k+1} and beta = G_k^+ W (W = Q_k^T Z_{k+1}).
// mixed != 0: convergence on the recursive residual only requests a
// true-residual refresh; the refresh decides.
template <int NB>
__device__ __forceinline__ void reduce_beta_body(Ctl* ctl, const double* part_rho, int nblk_rho,
                                                 const double* part_Wall, int nblk_W, int nwin, int cur,
                                                 const double* Gplus_all, double* beta_all, double* rhist,
                                                 int mixed) {
    // the state is tested after the reduction, so that its load and the
    // partial loads are in flight together (the partials are valid memory
    // whatever the state; with a stopped solve the sums are discarded)
    const int state = ctl->state;
    // slot j of W partials / G^+ / beta: part_Wall + j kMaxNB^2 nblk_W, + j kMaxNB^2
    const double* part_W = part_Wall + (size_t)cur * kMaxNB * kMaxNB * nblk_W;
    const double* Gplus = Gplus_all + (size_t)cur * kMaxNB * kMaxNB;
    double* beta = beta_all + (size_t)cur * kMaxNB * kMaxNB;
    __shared__ double red[1 + NB * NB];
    double* rho_s = red;
    double* W = red + 1;
    if constexpr (1 + NB * NB <= 40) {
        // ||r||^2 and W in one round of loads
        double v[1 + NB * NB];
        double v0[1], vW[NB * NB];
        partial_rows<1>(part_rho, nblk_rho, v0);
        partial_rows<NB * NB>(part_W, nblk_W, vW);
        v[0] = v0[0];
#pragma unroll
        for (int k = 0; k < NB * NB; ++k) v[1 + k] = vW[k];
        block_reduce<1 + NB * NB>(v, red);
    } else {
        reduce_partials<1>(part_rho, nblk_rho, rho_s);
        reduce_partials<NB * NB>(part_W, nblk_W, W);
    }
    if (state != 0) return;
    __shared__ int stop;
    if (threadIdx.x == 0) stop = beta_decide(ctl, rho_s[0], rhist, mixed);
    __syncthreads();
    if (stop) return;
    beta_apply<NB>(Gplus, W, beta, threadIdx.x, kRedBlock);
    // the other blocks of the window: beta_j = G_j^+ (Q_j^T Z)
    for (int j = 0; j < nwin; ++j) {
        if (j == cur) continue;
        __syncthreads();
        reduce_partials<NB * NB>(part_Wall + (size_t)j * kMaxNB * kMaxNB * nblk_W, nblk_W, W);
        beta_apply<NB>(Gplus_all + (size_t)j * kMaxNB * kMaxNB, W, beta_all + (size_t)j * kMaxNB * kMaxNB,
                       threadIdx.x, kRedBlock);
    }
}

template <int NB>
__global__ void __launch_bounds__(kRedBlock) k_reduce_beta(Ctl* ctl, const double* part_rho, int nblk_rho,
                                                        const double* part_Wall, int nblk_W, int nwin, int cur,
                                                        const double* Gplus_all, double* beta_all, double* rhist,
                                                        int mixed) {
    reduce_beta_body<NB>(ctl, part_rho, nblk_rho, part_Wall, nblk_W, nwin, cur, Gplus_all, beta_all, rhist, mixed);
}

// Gram G = P^T A P (upper triangle mirrored) and g = P^T r from the sums
// red[0 .. NG + NB) (shared), pseudo-inverse, alpha = G^+ g, rank; a rank of 0
// is a breakdown.  All threads of the block (at least 64) call it; G, Gp:
// shared NB x NB scratch, rank_s: a shared int.
template <int NB>
__device__ __forceinline__ void alpha_apply(Ctl* ctl, const double* red, double* G, double* Gp, int* rank_s,
                                            double* Gplus, double* alpha, double* ahist) {
    constexpr int NG = NB * (NB + 1) / 2;
    if (threadIdx.x == 0) {
        int q = 0;
        for (int a = 0; a < NB; ++a)
            for (int c = a; c < NB; ++c, ++q) G[a * NB + c] = G[c * NB + a] = red[q];
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        const int rk = wave_pinv<NB>(G, ctl->tau, Gp);
        if (threadIdx.x == 0) *rank_s = rk;
    }
    __syncthreads();
    if (threadIdx.x < NB * NB) Gplus[threadIdx.x] = Gp[threadIdx.x];
    if (threadIdx.x < NB) {
        double s = 0.0;
        for (int m = 0; m < NB; ++m) s += Gp[threadIdx.x * NB + m] * red[NG + m];
        alpha[threadIdx.x] = s;
        const int it = ctl->it;
        if (ahist && it < ctl->hist_cap) ahist[(size_t)it * NB + threadIdx.x] = s;
    }
    if (threadIdx.x == 0) {
        ctl->rank = *rank_s;
        if (*rank_s == 0) {
            ctl->status = kBREAKDOWN;
            ctl->state = 2;
        }
    }
}

// Gram G = P^T A P (upper triangle mirrored), g = P^T r, pseudo-inverse,
// alpha = G^+ g.  State 1 (stop after the x update) becomes 2 here.
template <int NB>
__device__ __forceinline__ void reduce_alpha_body(Ctl* ctl, const double* part, int nblk, double* Gplus,
                                                  double* alpha, double* ahist) {
    // the state is tested after the reduction, so that its load and the
    // partial loads are in flight together (see reduce_beta_body)
    const int state = ctl->state;
    constexpr int NG = NB * (NB + 1) / 2;
    __shared__ double red[NG + NB];
    __shared__ double G[NB * NB];
    __shared__ double Gp[NB * NB];
    __shared__ int rank_s;
    reduce_partials<NG + NB>(part, nblk, red);
    if (state == 2) return;
    if (state == 1) {
        if (threadIdx.x == 0) ctl->state = 2;
        return;
    }
    alpha_apply<NB>(ctl, red, G, Gp, &rank_s, Gplus, alpha, ahist);
}

template <int NB>
__global__ void __launch_bounds__(kRedBlock) k_reduce_alpha(Ctl* ctl, const double* part, int nblk, double* Gplus,
                                                         double* alpha, double* ahist) {
    reduce_alpha_body<NB>(ctl, part, nblk, Gplus, alpha, ahist);
}

// After a true-residual refresh r = b - A x: accept convergence or go on.
// One thread, given rho = ||b - A x||^2.
__device__ __forceinline__ void refresh_decide(Ctl* ctl, double rho, double* rhist) {
    ctl->refresh_req = 0;
    ctl->refreshes += 1;
    ctl->rho = rho;
    ctl->rho_ref = rho;
    const int it = ctl->it;
    if (rhist && it < ctl->hist_cap + 1) rhist[it] = sqrt(rho);
    if (!isfinite(rho)) {
        ctl->status = kNONFINITE;
        ctl->state = 2;
    } else if (rho <= ctl->tol2) {
        ctl->status = kOK;
        ctl->state = 2;
    }
}

__device__ __forceinline__ void refresh_reduce_body(Ctl* ctl, const double* part, int nblk, double* rhist) {
    if (ctl->state == 2 || !ctl->refresh_req) return;
    __shared__ double res[1];
    reduce_partials<1>(part, nblk, res);
    if (threadIdx.x != 0) return;
    refresh_decide(ctl, res[0], rhist);
}

static __global__ void __launch_bounds__(kRedBlock) k_refresh_reduce(Ctl* ctl, const double* part, int nblk, double* rhist) {
    refresh_reduce_body(ctl, part, nblk, rhist);
}

// Standalone pseudo-inverse of one Gram matrix (for the gram_pinv entry point).
template <int NB>
__global__ void __launch_bounds__(64) k_pinv_only(const double* G, double tau, double* Gplus, int* rank) {
    __shared__ double Gs[NB * NB];
    for (int q = threadIdx.x; q < NB * NB; q += 64) Gs[q] = G[q];
    __syncthreads();
    const int rk = wave_pinv<NB>(Gs, tau, Gplus);
    if (threadIdx.x == 0) *rank = rk;
}

}  // namespace amg
