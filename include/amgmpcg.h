/*
 * amgmpcg — additive-multigrid multipreconditioned CG on AMD MI355X (gfx950).
 *
 * C ABI of the solver library libamgmpcg.so.  Plain C types only: sizes are
 * int32/int64, arrays are raw pointers whose address space (host or device)
 * is stated per argument.  Every call returns an int status (AMGMPCG_OK or an
 * error code below); no C++ exception crosses this boundary.  A thread-local
 * text for the last error is available from amgmpcg_last_error().
 *
 * The method (Sec. 2 of the paper, Algorithm 1):
 *   r_0 = b - A x_0;  Z_k = [z^0 | ... | z^L] with z^l = P_l^L S_l^nu R_L^l r_k
 *   (the additive-multigrid correction of each level kept as its own search
 *   direction, coarsest first);  alpha = (P_k^T A P_k)^+ P_k^T r_k;
 *   x_{k+1} = x_k + P_k alpha;  r_{k+1} = r_k - A P_k alpha  (eq. (4));
 *   P_{k+1} = Z_{k+1} - sum_j P_j (P_j^T A P_j)^+ P_j^T A Z_{k+1} over the last
 *   m blocks j (truncation window m, option; m = 1: against P_k only).
 * S_l^nu is nu damped-Jacobi sweeps from zero (eq. (2)), R = 2^-d P^T (full
 * weighting), P tensor-product linear interpolation, A_l Galerkin products.
 *
 * Grid convention: unit square/cube, n interior nodes per axis, homogeneous
 * Dirichlet boundary, h = 1/(n+1); flat index i + n*(j + n*k) (x fastest).
 * Level l has floor(n / 2^(L-l)) nodes per axis; level L is the given grid.
 */
#ifndef AMGMPCG_H
#define AMGMPCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define AMGMPCG_OK            0   /* converged (relative residual <= tol)          */
#define AMGMPCG_MAXIT         1   /* iteration limit reached, x holds the iterate  */
#define AMGMPCG_BREAKDOWN     2   /* every direction dropped by the pseudo-inverse */
#define AMGMPCG_INVALID_ARG  -1   /* bad pointer, size or option                   */
#define AMGMPCG_NOT_SPD      -2   /* a level operator has a diagonal entry <= 0    */
#define AMGMPCG_DIM_MISMATCH -3   /* grid too small for the requested levels       */
#define AMGMPCG_NONFINITE    -4   /* NaN/Inf in the data or the residual           */
#define AMGMPCG_OOM          -5   /* device allocation failed                      */
#define AMGMPCG_HIP_ERROR    -6   /* any other HIP runtime error                   */
#define AMGMPCG_UNAVAILABLE  -7   /* entry point switched off in this build        */

/* ---- problem description -------------------------------------------- */
/* Structured diffusion problem -div(kappa grad u) = f on (0,1)^dim (eq. (1)
 * with K = kappa I, Dirichlet boundary), discretised by 5-/7-point finite
 * differences with harmonic-mean face coefficients 2 k_a k_b / (k_a + k_b).
 * kappa: HOST pointer to (n+2)^dim node values including the boundary layer
 * (x fastest), or NULL for kappa == 1 (Poisson).  Copied during setup. */
typedef struct {
    int32_t dim;        /* 2 or 3                                          */
    int32_t n;          /* interior nodes per axis, >= 1                   */
    int32_t nlevels;    /* levels including the finest, 1 <= nlevels <= 8  */
    const double* kappa;
} amgmpcg_grid;

/* A sparse matrix in CSR form (HOST arrays, copied during setup): row i
 * holds colind[rowptr[i] .. rowptr[i+1]-1] with values val[...]; indices
 * 0-based, int32; duplicates are summed. */
typedef struct {
    int32_t nrows, ncols, nnz;
    const int32_t* rowptr;   /* nrows + 1 entries, rowptr[0] = 0, rowptr[nrows] = nnz */
    const int32_t* colind;   /* nnz entries in [0, ncols)                            */
    const double* val;       /* nnz entries                                          */
} amgmpcg_csr;

/* A nested hierarchy given by its prolongations (Sec. 2.1 with arbitrary
 * transfers): P[l] maps level l to level l+1 (P[l].nrows = unknowns of
 * level l+1, P[l].ncols = unknowns of level l; level 0 coarsest, level
 * nlevels-1 the finest), R_l = restrict_scale * P[l]^T. */
typedef struct {
    int32_t nlevels;           /* 1..8                                      */
    const amgmpcg_csr* P;      /* HOST array of nlevels - 1 matrices (NULL if nlevels = 1) */
    double restrict_scale;     /* > 0                                       */
} amgmpcg_hierarchy;

/* Solver options.  Fill with amgmpcg_default_options() first. */
typedef struct {
    int32_t m;            /* truncation window 1..8 (1): P_{k+1} is made
                             A-orthogonal to the last m direction blocks
                             (classical Gram-Schmidt, every beta_j from Z);
                             the blocks and their Q = A P are kept in a ring */
    int32_t nu;           /* damped-Jacobi sweeps on every level, 1..8 (2)     */
    double  omega;        /* Jacobi damping in (0, 1] (2/3)                   */
    int32_t maxit;        /* iteration limit (1000)                            */
    int32_t precision;    /* 0: FP64 throughout; 1: FP32 bulk (operators,
                             transfers, smoothers, direction blocks) with FP64
                             x, r, Gram, pseudo-inverse and residual refresh */
    double  pinv_tau;     /* eigenvalue cut of the unit-diagonal Gram; <= 0:
                             64 * b * u with u = 2^-53 (FP64) or 2^-24 (FP32) */
    int32_t k_poll;       /* iterations per captured graph launch between
                             host checks of the device stop flag (8)          */
    int32_t record_history; /* keep alpha and ||r|| per iteration (1)          */
    double  refresh_drop; /* FP32 bulk: replace r by b - A x (FP64) whenever
                             ||r|| fell by this factor since the last refresh,
                             and before accepting convergence (1e-2)          */
    int32_t method;       /* AMGMPCG_METHOD_*: the solver of Algorithm 1 (0)
                             or one of the comparison methods of Sec. 3, CG
                             with one search direction per iteration         */
    int32_t nu_pre;       /* V-cycle (method 2): damped-Jacobi sweeps before
                             and after the coarse correction on every level
                             but the coarsest, which gets nu_pre + nu_post
                             from zero; 0: max(1, nu / 2).  Must be equal
                             (a symmetric preconditioner for CG)            */
    int32_t nu_post;
    int32_t true_residual; /* 1: every solve also computes the true relative
                             residual ||b - A x||_2 / ||b||_2 of the returned
                             x with the FP64 finest operator (one more
                             operator application and norm, part of the
                             solve's device time) into info->relres_true;
                             0: not computed (relres_true = -1)  (1)     */
    int32_t persistent;   /* batched handles: 1 = the whole solve of every
                             problem in one persistent launch (each workgroup
                             runs Algorithm 1 for one problem at a time,
                             problems taken largest first from a queue);
                             0 = one batched launch per step of Algorithm 1
                             over all problems, k_poll iterations per graph
                             (0: the faster form on MI355X)                 */
} amgmpcg_options;

/* Solution methods (amgmpcg_options.method).  The comparison methods share
 * the hierarchy, smoother, transfers and the SpMM/Gram and reduction kernels
 * of the MPCG solver; they need m = 1 and no learned direction. */
#define AMGMPCG_METHOD_MPCG          0  /* Algorithm 1: the L+1 level
                                           corrections as separate directions */
#define AMGMPCG_METHOD_ADDITIVE_PCG  1  /* CG preconditioned by the sum of the
                                           level corrections (eq. (3))        */
#define AMGMPCG_METHOD_VCYCLE_PCG    2  /* CG preconditioned by one V-cycle
                                           (multiplicative MG, Sec. 2.1)      */

typedef struct {
    int32_t status;          /* AMGMPCG_OK / _MAXIT / _BREAKDOWN / _NONFINITE   */
    int32_t iterations;      /* number of x updates                             */
    double  bnorm;           /* ||b||_2                                         */
    double  relres;          /* last ||r||_2 / ||b||_2 on the solver's r        */
    int32_t refreshes;       /* FP32 bulk: true-residual refreshes performed   */
    int32_t nb;              /* search directions per iteration (L + 1, or L + 2
                                with the learned direction)                     */
    double  solve_ms;        /* device time of the solve (HIP events)           */
    double  relres_true;     /* ||b - A x||_2 / ||b||_2 of the returned x in FP64
                                (options.true_residual = 1), else -1; -1 for
                                batched solves                                  */
    double  setup_ms;        /* host wall time of the handle's setup call       */
} amgmpcg_info;

typedef struct amgmpcg_handle amgmpcg_handle;

/* Default options (m=1, nu=2, omega=2/3, maxit=1000, FP64, k_poll=8,
 * method MPCG, nu_pre = nu_post = 0, true_residual = 1, persistent = 0). */
void amgmpcg_default_options(amgmpcg_options* opts);

/* setup(A, hierarchy): build the level hierarchy of a structured problem.
 * Level operators are Galerkin products A_l = R A_{l+1} P computed on the
 * host (Sec. 2.1), stored symmetrised, checked for a positive diagonal
 * (AMGMPCG_NOT_SPD otherwise) and uploaded.  stream: hipStream_t on which
 * every device operation of this handle runs (NULL = default stream).  The
 * handle owns all device memory it allocates; free with amgmpcg_destroy. */
int amgmpcg_setup_grid(const amgmpcg_grid* grid, const amgmpcg_options* opts,
                       void* stream, amgmpcg_handle** out);

/* setup(A, hierarchy) for a general SPD matrix and hierarchy (Sec. 2.1):
 * A (nrows = ncols = n) and the prolongations of H, all HOST CSR, copied.
 * The coarse operators are the Galerkin products R_l A_{l+1} P_l built on
 * the host (stored symmetrised: upper triangle mirrored), the smoother is
 * the damped Jacobi of every level; the solve runs Algorithm 1 with CSR
 * kernels (one thread per row).  Options as for amgmpcg_setup_grid with the
 * MPCG method only.  Errors (before any device call): AMGMPCG_INVALID_ARG
 * for malformed CSR data (row pointers, index ranges, nnz) or dimensions
 * that do not chain, AMGMPCG_NONFINITE for non-finite values,
 * AMGMPCG_NOT_SPD for a non-symmetric A (relative 1e-12) or a non-positive
 * diagonal on any level; then AMGMPCG_OOM / AMGMPCG_HIP_ERROR.  Entry points
 * tied to structured grids or the learned direction (level_stencil,
 * attach_cnn, log_kappa, make_pairs, time_kernels, profile_solve) return
 * AMGMPCG_INVALID_ARG for such a handle; amgmpcg_level_size gives a level's
 * number of unknowns. */
int amgmpcg_setup_csr(const amgmpcg_csr* A, const amgmpcg_hierarchy* H, const amgmpcg_options* opts,
                      void* stream, amgmpcg_handle** out);

/* setup(A, hierarchy) for a 2D operator given by a constant 9-point stencil
 * on the finest level (Sec. 3, Example 1: bilinear finite elements for
 * anisotropic diffusion on a uniform mesh), the rest as amgmpcg_setup_grid
 * (the same nested grids, transfers and Galerkin coarse operators).
 * grid: dim must be 2 and kappa NULL; n interior nodes per axis (m = n + 1
 * elements).  stencil: HOST, 9 doubles, stencil[(dy+1)*3 + (dx+1)] =
 * A(idx, idx + dx + n dy) at interior nodes, couplings to the boundary
 * dropped (homogeneous Dirichlet); it must be symmetric
 * (stencil[q] == stencil[8-q]) with a positive centre.  Errors:
 * AMGMPCG_INVALID_ARG, AMGMPCG_NONFINITE, AMGMPCG_NOT_SPD (before any device
 * call), AMGMPCG_OOM / AMGMPCG_HIP_ERROR. */
int amgmpcg_setup_stencil(const amgmpcg_grid* grid, const double* stencil, const amgmpcg_options* opts,
                          void* stream, amgmpcg_handle** out);

/* solve(b, x0, tol): Algorithm 1 until ||r_k||_2 <= tol ||b||_2 or maxit.
 * b_dev: DEVICE pointer, n^dim doubles, read only.  x_dev: DEVICE pointer,
 * n^dim doubles, x_0 on entry and the final iterate on return.  Both are
 * used on the handle's stream and not retained after the call returns.
 * maxit <= 0 uses the option value.  tol = 0 runs exactly maxit iterations
 * (unless the residual vanishes).  info may be NULL.  Returns the solve
 * status (also in info->status). */
int amgmpcg_solve(amgmpcg_handle* h, const double* b_dev, double* x_dev,
                  double tol, int32_t maxit, amgmpcg_info* info);

/* As amgmpcg_solve with HOST b and x (copies over PCIe included). */
int amgmpcg_solve_host(amgmpcg_handle* h, const double* b, double* x,
                       double tol, int32_t maxit, amgmpcg_info* info);

/* The block Z = [z^0 | ... | z^L] of level corrections of r (Algorithm 1,
 * "corrections from all levels").  r_dev: DEVICE, n^dim doubles.  Z_dev:
 * DEVICE, column-major n^dim x (L+1) doubles (column l = level l, coarsest
 * first), written in the handle's precision and widened to double.
 * AMGMPCG_INVALID_ARG for a handle set up with a comparison method. */
int amgmpcg_mg_block(amgmpcg_handle* h, const double* r_dev, double* Z_dev);

/* Number of levels, search directions and per-axis nodes of level l. */
int amgmpcg_level_count(const amgmpcg_handle* h, int32_t* nlevels, int32_t* nb);
int amgmpcg_level_size(const amgmpcg_handle* h, int32_t level, int32_t* n_axis);

/* The operator of a coarse level l < L as 3^dim stencil coefficients per node,
 * HOST out array of 3^dim * n_l^dim doubles, out[s * N_l + i] = A_l(i, i+o_s)
 * with o_s = (dx,dy,dz) and s = (dz+1)*9 + (dy+1)*3 + (dx+1) (2D: no dz
 * term); entries whose neighbour lies outside the grid are 0. */
int amgmpcg_level_stencil(const amgmpcg_handle* h, int32_t level, double* out);

/* Per-iteration history of the last solve (record_history = 1): alpha_out
 * (HOST, cap * nb doubles, row k = alpha_k) and resnorm_out (HOST, cap + 1
 * doubles, ||r_k||_2).  Either may be NULL.  *count = iterations stored. */
int amgmpcg_history(const amgmpcg_handle* h, int32_t cap, double* alpha_out,
                    double* resnorm_out, int32_t* count);

/* Batched solves: count independent Poisson problems (kappa must be NULL,
 * all of one dim, each with its own n and nlevels <= 6) whose hierarchies
 * are built here (Sec. 2.1 per problem); grids: HOST array of count entries.
 * opts as for amgmpcg_setup_grid (nu must be 1 or 2, m = 1, the MPCG
 * method).  The problems are solved together (Algorithm 1 for each), each
 * with its own convergence flag.  With opts->persistent = 0 (default) every
 * step is one launch over all problems with the same number of levels, each
 * block working on one problem's nodes, and k_poll iterations of all
 * problems are captured in one HIP graph, launched until every problem has
 * stopped.  With opts->persistent = 1 one persistent launch, captured in a
 * HIP graph with the reset of its work queue, runs every problem's whole
 * solve: each workgroup of 512 threads takes the next problem (largest
 * first), runs all iterations of Algorithm 1 for it with workgroup-wide
 * reductions and barriers between the steps, and takes the next, until none
 * is left.  Both forms give the same iterates up to rounding order.  Errors: AMGMPCG_INVALID_ARG for bad arguments (checked before
 * any device call), AMGMPCG_NOT_SPD, AMGMPCG_OOM / AMGMPCG_HIP_ERROR from
 * the device. */
int amgmpcg_setup_batched(int32_t count, const amgmpcg_grid* grids, const amgmpcg_options* opts,
                          void* stream, amgmpcg_handle** out);

/* b_dev, x_dev: DEVICE, the problems' vectors concatenated in the order of
 * grids (problem i starts at offset sum_{j<i} n_j^dim); x holds every x_0 on
 * entry and every result on return.  infos: HOST, count entries or NULL.
 * batch_ms: device time of the whole solve (HIP events) or NULL.  Returns
 * AMGMPCG_OK if every problem converged, else the first other status. */
int amgmpcg_solve_batched(amgmpcg_handle* h, const double* b_dev, double* x_dev, double tol,
                          int32_t maxit, amgmpcg_info* infos, double* batch_ms);

/* Number of problems and total unknowns of a batched handle. */
int amgmpcg_batched_size(const amgmpcg_handle* h, int32_t* count, int64_t* total_dofs);

/* Device memory a handle holds, in bytes.  For a handle of setup_grid,
 * setup_stencil or setup_csr: the bytes of a caller workspace that holds all
 * of the handle's device buffers (level operators and transfers, vectors,
 * direction blocks and their rings, partial sums, history; with an attached
 * network also its wider blocks), each at a 256-byte aligned offset: the
 * size amgmpcg_bind_workspace needs.  Not counted: a few hundred bytes of
 * control words and the captured iteration graph, which the handle always
 * owns.  For a batched handle: the bytes its setup allocated.  A solve
 * allocates nothing except on a handle's first solve (after setup or a
 * bind), which captures the iteration graph.  The network's own buffers
 * belong to the network.  Errors: INVALID_ARG for a NULL handle or output
 * pointer. */
int amgmpcg_workspace_bytes(const amgmpcg_handle* h, int64_t* bytes);

/* Route the device buffers of a handle through caller-owned device memory
 * (for example a torch tensor), in the spirit of Algorithm 1's problem
 * statement: the caller provides all storage of the iteration.
 * device_ptr: DEVICE memory of at least amgmpcg_workspace_bytes(h) bytes,
 * 256-byte aligned.  Every buffer of the handle is copied into it (on the
 * handle's stream; the call synchronises), the handle's own copies are
 * freed, and the next solve captures the iteration graph anew.  From then
 * on the caller owns the memory: it must stay allocated, and must not be
 * written, while the handle exists; amgmpcg_destroy does not free it.
 * Binding again moves the buffers to the new region (the old one may then
 * be released).  Results are bit for bit those of the unbound handle.
 * Attach or detach a network (amgmpcg_attach_cnn) before binding.  Errors,
 * checked on the host before any copy: AMGMPCG_INVALID_ARG for a NULL or
 * batched handle, a NULL, host or unaligned pointer, or bytes below the
 * need; then AMGMPCG_HIP_ERROR for a failed copy. */
int amgmpcg_bind_workspace(amgmpcg_handle* h, void* device_ptr, int64_t bytes);

/* Measurement aid: average duration in ms of each hot kernel of one
 * iteration, each launched reps times back to back between two HIP events
 * on the handle's stream, on the state left by the last solve (call it after
 * a solve; it overwrites the solver's work vectors, not the caller's x).
 * ms_out: HOST, cap doubles, in the order update_r, fine_smooth,
 * restrict_fine, coarse_smooth, prolong_top, fine_W, update_xP, spmm_gram,
 * residual (9 entries; 0 where a level does not exist). *count = entries. */
int amgmpcg_time_kernels(amgmpcg_handle* h, int32_t reps, double* ms_out, int32_t cap, int32_t* count);

/* Measurement aid: amgmpcg_solve with the iterations launched one by one
 * (no graph) and HIP events between the kernel groups of each iteration, so
 * every kernel runs on the data the previous one just wrote.  ms_out (HOST,
 * cap doubles) receives the average duration in ms, over the iterations
 * that ran in full (*samples of them; the last iteration, whose SpMM and
 * alpha step the stop flag skips, is left out), of: update_r, fine_smooth,
 * restrict, coarse_smooth, prolong, learned, fine_W, reduce_beta,
 * update_xP, refresh, spmm_gram, reduce_alpha, whole iteration, and the
 * x/P update kernel alone (14 entries, *count = 14; 0 for a group that does
 * not run).  The groups are spans between events recorded on the stream, so
 * they include the launch latency; the last entry comes from events bound
 * to the x/P update's dispatch itself (hipExtLaunchKernel start and stop
 * events), the kernel's own duration.  b, x, tol, maxit and the result as
 * for amgmpcg_solve (info->solve_ms = 0). */
int amgmpcg_profile_solve(amgmpcg_handle* h, const double* b_dev, double* x_dev, double tol, int32_t maxit,
                          amgmpcg_info* info, double* ms_out, int32_t cap, int32_t* count, int32_t* samples);

/* The device pseudo-inverse used for the step coefficients (Sec. 2.2: the
 * Gram P^T A P may be singular), applied to one symmetric positive
 * semi-definite nb x nb matrix.  G, Gplus: HOST, nb*nb doubles row-major.
 * Columns with a non-positive or non-finite diagonal are inactive; on the
 * unit-diagonal scaling Ghat = S G S eigenvalues <= tau are dropped and
 * Gplus = S Ghat^+ S.  *rank = eigenvalues kept.  Runs on the default
 * stream and synchronises. */
int amgmpcg_gram_pinv(const double* G, int32_t nb, double tau, double* Gplus, int32_t* rank);

/* amgmpcg_gram_pinv for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernel and result, with the device staging of G, G^+
 * and the rank in a static device array of the library (1 KiB on every GPU
 * it runs on, held until the process ends) instead of a buffer allocated per
 * call; no hipMalloc, hipFree or other allocating call.  nb is limited to
 * 1..8 (the array holds an 8 x 8 Gram); larger nb returns
 * AMGMPCG_INVALID_ARG.  Every call on one GPU uses that GPU's one array:
 * calls that overlap on one GPU (from several host threads) race.  Runs on
 * the default stream of the current device and synchronises. */
int amgmpcg_gram_pinv_noalloc(const double* G, int32_t nb, double tau, double* Gplus, int32_t* rank);

/* r = b - A x with the finest operator in FP64.  b_dev, x_dev, r_dev:
 * DEVICE, n^dim doubles each (r may not alias b or x). */
int amgmpcg_residual(amgmpcg_handle* h, const double* b_dev, const double* x_dev, double* r_dev);

/* ---- learned search direction --------------------------------------- */
/* A convolutional network N (a 3-level U-Net: 3x3x3 convolutions without
 * bias, ReLU, 2x2x2 average pooling, nearest upsampling with skip
 * concatenation, 16/32/64 channels, a 1x1x1 output convolution) maps a
 * residual r to an approximation of the error; its output is appended to the
 * block Z of Algorithm 1 as one more column, so that the energy minimisation
 * over span(P_k) chooses its coefficient (and can set it to zero).  Inputs:
 * channel 0 = r / rms(r), channel 1 = log kappa at the nodes normalised to
 * zero mean and unit standard deviation (0 for Poisson).  The network runs
 * on an S^3 grid, S = n rounded up to a multiple of 4, holding the n^3 nodes
 * in its low corner and zeros elsewhere.  Weights, activations and their
 * gradients are bfloat16 with FP32 accumulation on the matrix cores; the
 * FP32 master weights are trained with Adam on the device.  3D only. */
typedef struct amgmpcg_cnn amgmpcg_cnn;

/* Number of FP32 weights.  Layout: layers w1..w11 in order, each
 * [tap][Cout][Cin] row-major with tap t = (dz+1)*9 + (dy+1)*3 + (dx+1)
 * (one tap for w11), layer shapes (Cin -> Cout): w1 16->16 (input channels
 * 2..15 are zero), w2 16->16, w3 16->32, w4 32->32, w5 32->64, w6 64->64,
 * w7 96->32, w8 32->32, w9 48->16, w10 16->16, w11 16->16 (only output
 * channel 0 is used). */
int64_t amgmpcg_cnn_weight_count(void);

/* A network for n^3 problem grids (1 <= n <= 1000) with He-normal initial
 * weights from seed; stream: hipStream_t of every operation (NULL = the
 * default stream).  The network owns its device memory; one network serves
 * one call at a time. */
int amgmpcg_cnn_create(int32_t n, uint64_t seed, void* stream, amgmpcg_cnn** out);

/* Weights, HOST, count = amgmpcg_cnn_weight_count() floats.  set_weights
 * also resets the Adam moments and step count. */
int amgmpcg_cnn_set_weights(amgmpcg_cnn* net, const float* w, int64_t count);
int amgmpcg_cnn_get_weights(amgmpcg_cnn* net, float* w, int64_t count);
/* Weight gradients of the last amgmpcg_cnn_gradients/train_step call. */
int amgmpcg_cnn_get_gradients(amgmpcg_cnn* net, float* g, int64_t count);

/* d = N(r).  r_dev, d_dev: DEVICE, n^3 doubles.  lk_dev: DEVICE, n^3
 * bfloat16 bit patterns of the normalised log kappa (amgmpcg_log_kappa), or
 * NULL for zeros.  Returns AMGMPCG_NONFINITE if d has a NaN/Inf (d is
 * still written). */
int amgmpcg_cnn_forward(amgmpcg_cnn* net, const double* r_dev, const uint16_t* lk_dev, double* d_dev);

/* Loss and gradients for one training pair (r, e) with e the error x* - x
 * that left residual r: loss = mean over the n^3 nodes of
 * (N(r) - e / rms(e))^2.  r_dev, e_dev: DEVICE, n^3 doubles; lk_dev as for
 * forward.  *loss (HOST) receives the loss of the forward pass.
 * train_step additionally applies one Adam step (beta1 0.9, beta2 0.999,
 * eps 1e-8) with learning rate lr > 0 to the FP32 masters. */
int amgmpcg_cnn_gradients(amgmpcg_cnn* net, const double* r_dev, const uint16_t* lk_dev,
                          const double* e_dev, double* loss);
int amgmpcg_cnn_train_step(amgmpcg_cnn* net, const double* r_dev, const uint16_t* lk_dev,
                           const double* e_dev, float lr, double* loss);

/* One training step on the energy loss of the direction d = N(r):
 * marginal = 0: loss = 1 - (d.r)^2 / ((d.A d)(e.r)), the fraction of the
 * squared A-norm error ||e||_A^2 = e.r left by the best step along d alone
 * (A: the finest operator of handle h, whose grid must equal the network's;
 * e.r uses A e = r).  marginal = 1: the same with r and A d replaced by their
 * parts A-orthogonal to the level-correction block Z = MG(r) of h (r^ = r - A
 * Z alpha after the energy-minimising step over Z, A d^ = A d - A Z G^+ Z^T A
 * d): the fraction of the error left by the step over Z that stays after
 * adding d (h must be FP64 with no network attached; its work vectors are
 * overwritten).  Scale-free in d.  lr > 0 applies one Adam step, lr = 0 only
 * computes the gradients.  Arguments as for amgmpcg_cnn_train_step. */
int amgmpcg_cnn_energy_step(amgmpcg_cnn* net, amgmpcg_handle* h, const double* r_dev, const uint16_t* lk_dev,
                            const double* e_dev, int32_t marginal, float lr, double* loss);

/* The energy loss of amgmpcg_cnn_energy_step for a given direction d (no
 * network) and its gradient dL/dd in FP64, on the default stream
 * (synchronises).  d_dev, r_dev, e_dev, grad_dev: DEVICE, n^dim doubles;
 * *loss: HOST.  marginal = 1 overwrites the handle's work vectors. */
int amgmpcg_energy_grad(amgmpcg_handle* h, const double* d_dev, const double* r_dev, const double* e_dev,
                        int32_t marginal, double* grad_dev, double* loss);

/* Average time in ms of one inference (reps back-to-back forward passes
 * between two HIP events on the network's stream).  ms: HOST. */
int amgmpcg_cnn_time_forward(amgmpcg_cnn* net, const double* r_dev, const uint16_t* lk_dev,
                             int32_t reps, double* ms);

/* One layer l (0..10 for w1..w11) of the network, with its current
 * weights, on caller tensors: channels-last bfloat16 bit patterns on an S^3
 * grid (1 <= S <= 512), zero outside the grid.
 *   op 0: out = relu(conv_l(A)), bfloat16 with Cout channels (l = 10: no
 *         ReLU, FP32 output channel 0 only, one value per voxel);
 *   op 1: out = conv_l^T(A): the data gradient for an output gradient A
 *         (Cout channels), bfloat16 with Cin channels;
 *   op 2: out = the weight gradient for output gradient A (Cout channels)
 *         and layer input B (Cin channels): FP32 [tap][Cout][Cin].
 * A_dev, B_dev, out_dev: DEVICE.  Synchronises. */
int amgmpcg_cnn_layer(amgmpcg_cnn* net, int32_t layer, int32_t op, int32_t S, const uint16_t* A_dev,
                      const uint16_t* B_dev, void* out_dev);

/* Free a network.  Detach it from every handle first. */
void amgmpcg_cnn_destroy(amgmpcg_cnn* net);

/* Append the learned direction N(r_k) to every block Z_k of the solves of
 * this 3D handle (net = NULL removes it).  nb becomes nlevels + 1 (needs
 * nlevels <= 7); a direction with a NaN/Inf value is replaced by zero, which
 * the pseudo-inverse then drops.  The handle keeps the pointer: the network
 * must outlive the attachment.  AMGMPCG_DIM_MISMATCH if the network's n
 * differs from the grid's. */
int amgmpcg_attach_cnn(amgmpcg_handle* h, amgmpcg_cnn* net);

/* The network's second input channel for this handle's kappa: DEVICE out,
 * n^3 bfloat16 bit patterns (zeros for Poisson). */
int amgmpcg_log_kappa(amgmpcg_handle* h, uint16_t* lk_dev);

/* Training pairs from this handle's iteration: for each k = ks[i] (HOST,
 * nk entries, k >= 0), x_k = k iterations of amgmpcg_solve from x_0 = 0
 * with tol = 0, R_dev[i*N ..] = b - A x_k and E_dev[i*N ..] = xs - x_k
 * (N = n^dim; DEVICE, nk*N doubles each; xs_dev the converged solution).
 * Uses the attached network if any. */
int amgmpcg_make_pairs(amgmpcg_handle* h, const double* b_dev, const double* xs_dev, const int32_t* ks,
                       int32_t nk, double* R_dev, double* E_dev);

void amgmpcg_destroy(amgmpcg_handle* h);
const char* amgmpcg_status_string(int status);
const char* amgmpcg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* AMGMPCG_H */
