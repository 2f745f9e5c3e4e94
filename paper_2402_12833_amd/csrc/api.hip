// libamgmpcg: additive-multigrid MPCG (Algorithm 1 of the paper) on gfx950.
//
// The extern "C" entry points declared in include/amgmpcg.h: argument
// validation on the host, the handle, and dispatch to the solver types
// (each in its own translation unit) and to the learned direction.
#include <mutex>

#include "host_common.hpp"
#include "cnn_host.hpp"

namespace amg {

thread_local std::string g_last_error;
thread_local int64_t g_devbuf_bytes = 0;

// Device staging of amgmpcg_gram_pinv_noalloc: G (kMaxNB^2 doubles), G^+
// (kMaxNB^2) and the rank, in a file-scope device array that every GPU the
// library runs on holds until the process ends.  In host code its name is a
// host-side stand-in: kernels and copies use the address from
// hipGetSymbolAddress, looked up once per device.
constexpr int kPinvScratch = 2 * kMaxNB * kMaxNB + 8;
static __device__ __align__(256) double scratch[kPinvScratch];
constexpr int kMaxDevices = 64;
static double* g_scratch_dev[kMaxDevices];
static std::mutex g_scratch_mu;

// The current device's address of the staging array.
static double* pinv_scratch() {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) throw ApiError(AMGMPCG_INVALID_ARG, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) throw ApiError(AMGMPCG_HIP_ERROR, "no device address for the staging array");
        g_scratch_dev[dev] = static_cast<double*>(ptr);
    }
    return g_scratch_dev[dev];
}

// One pseudo-inverse of an nb x nb Gram matrix at device G (kernel k_pinv_only).
static void launch_pinv(int nb, const double* G, double tau, double* Gplus, int* rank) {
    switch (nb) {
        case 1: k_pinv_only<1><<<1, 64>>>(G, tau, Gplus, rank); break;
        case 2: k_pinv_only<2><<<1, 64>>>(G, tau, Gplus, rank); break;
        case 3: k_pinv_only<3><<<1, 64>>>(G, tau, Gplus, rank); break;
        case 4: k_pinv_only<4><<<1, 64>>>(G, tau, Gplus, rank); break;
        case 5: k_pinv_only<5><<<1, 64>>>(G, tau, Gplus, rank); break;
        case 6: k_pinv_only<6><<<1, 64>>>(G, tau, Gplus, rank); break;
        case 7: k_pinv_only<7><<<1, 64>>>(G, tau, Gplus, rank); break;
        default: k_pinv_only<8><<<1, 64>>>(G, tau, Gplus, rank); break;
    }
    HIPCHK(hipGetLastError());
}

SolverBase* new_grid_solver_d2(const amgmpcg_grid&, const amgmpcg_options&, hipStream_t, const double*);
SolverBase* new_grid_solver_d3(const amgmpcg_grid&, const amgmpcg_options&, hipStream_t, const double*);
SolverBase* new_grid_solver_f2(const amgmpcg_grid&, const amgmpcg_options&, hipStream_t, const double*);
SolverBase* new_grid_solver_f3(const amgmpcg_grid&, const amgmpcg_options&, hipStream_t, const double*);

SolverBase* new_grid_solver(int precision, int dim, const amgmpcg_grid& g, const amgmpcg_options& o,
                            hipStream_t stream, const double* st9) {
    if (precision == 0) return dim == 2 ? new_grid_solver_d2(g, o, stream, st9) : new_grid_solver_d3(g, o, stream, st9);
    return dim == 2 ? new_grid_solver_f2(g, o, stream, st9) : new_grid_solver_f3(g, o, stream, st9);
}

namespace cnn {
void net_forward(Net& net, const Ctl* ctl, const double* r, const bf16* lk, hipStream_t s) {
    net.forward(ctl, r, lk, s);
}
}  // namespace cnn

}  // namespace amg

struct amgmpcg_handle {
    std::unique_ptr<amg::SolverBase> s;
    std::unique_ptr<amg::BatchedBase> bs;
    int64_t bytes = 0;   // device buffers allocated at setup and by attach
    double setup_ms = 0.0;   // host wall time of the setup call
};

// Host wall time since t0 in ms.
static double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

struct amgmpcg_cnn {
    amg::cnn::Net net;
};

using amg::ApiError;

template <typename F>
static int guarded(F&& f) {
    try {
        amg::g_last_error.clear();
        return f();
    } catch (const ApiError& e) {
        amg::g_last_error = e.what();
        return e.code;
    } catch (const std::bad_alloc&) {
        amg::g_last_error = "host out of memory";
        return AMGMPCG_OOM;
    } catch (const std::exception& e) {
        amg::g_last_error = e.what();
        return AMGMPCG_HIP_ERROR;
    }
}

static void validate_options(const amgmpcg_options* o) {
    if (!o) throw ApiError(AMGMPCG_INVALID_ARG, "options pointer is NULL");
    if (o->m < 1 || o->m > amg::kMaxWin) throw ApiError(AMGMPCG_INVALID_ARG, "m must be in 1..8");
    if (o->nu < 1 || o->nu > 8) throw ApiError(AMGMPCG_INVALID_ARG, "nu must be in 1..8");
    if (!(o->omega > 0.0 && o->omega <= 1.0)) throw ApiError(AMGMPCG_INVALID_ARG, "omega must be in (0, 1]");
    if (o->maxit < 1) throw ApiError(AMGMPCG_INVALID_ARG, "maxit must be >= 1");
    if (o->precision != 0 && o->precision != 1) throw ApiError(AMGMPCG_INVALID_ARG, "precision must be 0 or 1");
    if (o->k_poll < 1 || o->k_poll > 64) throw ApiError(AMGMPCG_INVALID_ARG, "k_poll must be in 1..64");
    if (!(o->refresh_drop > 0.0 && o->refresh_drop < 1.0))
        throw ApiError(AMGMPCG_INVALID_ARG, "refresh_drop must be in (0, 1)");
    if (o->method < AMGMPCG_METHOD_MPCG || o->method > AMGMPCG_METHOD_VCYCLE_PCG)
        throw ApiError(AMGMPCG_INVALID_ARG, "method must be 0, 1 or 2");
    if (o->method != AMGMPCG_METHOD_MPCG && o->m != 1)
        throw ApiError(AMGMPCG_INVALID_ARG, "the comparison methods need m = 1");
    if (o->nu_pre < 0 || o->nu_pre > 8 || o->nu_post < 0 || o->nu_post > 8)
        throw ApiError(AMGMPCG_INVALID_ARG, "nu_pre and nu_post must be in 0..8");
    if (o->nu_pre != o->nu_post)
        throw ApiError(AMGMPCG_INVALID_ARG, "nu_pre and nu_post must be equal (symmetric V-cycle)");
    if (o->true_residual != 0 && o->true_residual != 1)
        throw ApiError(AMGMPCG_INVALID_ARG, "true_residual must be 0 or 1");
    if (o->persistent != 0 && o->persistent != 1) throw ApiError(AMGMPCG_INVALID_ARG, "persistent must be 0 or 1");
}

static void validate_grid(const amgmpcg_grid* g) {
    if (!g) throw ApiError(AMGMPCG_INVALID_ARG, "grid pointer is NULL");
    if (g->dim != 2 && g->dim != 3) throw ApiError(AMGMPCG_INVALID_ARG, "dim must be 2 or 3");
    if (g->n < 1) throw ApiError(AMGMPCG_INVALID_ARG, "n must be >= 1");
    if (g->nlevels < 1 || g->nlevels > amg::kMaxNB) throw ApiError(AMGMPCG_INVALID_ARG, "nlevels must be in 1..8");
    const double total = std::pow((double)g->n, g->dim);
    if (total > 1.0e9) throw ApiError(AMGMPCG_INVALID_ARG, "grid too large");
    int n = g->n;
    for (int l = 1; l < g->nlevels; ++l) {
        n /= 2;
        if (n < 1) throw ApiError(AMGMPCG_DIM_MISMATCH, "grid too small for the requested number of levels");
    }
    if (g->kappa) {
        const int64_t m = (int64_t)std::llround(std::pow((double)(g->n + 2), g->dim));
        for (int64_t i = 0; i < m; ++i) {
            const double k = g->kappa[i];
            if (!std::isfinite(k)) throw ApiError(AMGMPCG_NONFINITE, "kappa has a non-finite value");
            if (!(k > 0.0)) throw ApiError(AMGMPCG_NOT_SPD, "kappa must be positive");
        }
    }
}

extern "C" {

void amgmpcg_default_options(amgmpcg_options* o) {
    if (!o) return;
    o->m = 1;
    o->nu = 2;
    o->omega = 2.0 / 3.0;
    o->maxit = 1000;
    o->precision = 0;
    o->pinv_tau = 0.0;
    o->k_poll = 8;
    o->record_history = 1;
    o->refresh_drop = 1e-2;
    o->method = AMGMPCG_METHOD_MPCG;
    o->nu_pre = 0;
    o->nu_post = 0;
    o->true_residual = 1;
    o->persistent = 0;
}

int amgmpcg_setup_grid(const amgmpcg_grid* grid, const amgmpcg_options* opts, void* stream, amgmpcg_handle** out) {
    return guarded([&]() -> int {
        if (!out) throw ApiError(AMGMPCG_INVALID_ARG, "out pointer is NULL");
        *out = nullptr;
        validate_grid(grid);
        validate_options(opts);
        const auto t0 = std::chrono::steady_clock::now();
        auto h = std::make_unique<amgmpcg_handle>();
        const int64_t bytes0 = amg::g_devbuf_bytes;
        hipStream_t s = (hipStream_t)stream;
        h->s.reset(amg::new_grid_solver(opts->precision, grid->dim, *grid, *opts, s, nullptr));
        h->bytes = amg::g_devbuf_bytes - bytes0;
        h->setup_ms = ms_since(t0);
        *out = h.release();
        return AMGMPCG_OK;
    });
}

// A HOST CSR matrix checked and copied (duplicates summed by the products).
static amg::host::Csr csr_copy(const amgmpcg_csr* M, const char* what) {
    if (!M) throw ApiError(AMGMPCG_INVALID_ARG, std::string(what) + " is NULL");
    if (M->nrows < 1 || M->ncols < 1 || M->nnz < 0 || !M->rowptr || (M->nnz > 0 && (!M->colind || !M->val)))
        throw ApiError(AMGMPCG_INVALID_ARG, std::string(what) + ": bad dimensions or NULL arrays");
    if (M->rowptr[0] != 0 || M->rowptr[M->nrows] != M->nnz)
        throw ApiError(AMGMPCG_INVALID_ARG, std::string(what) + ": row pointers do not span nnz");
    amg::host::Csr C;
    C.n = M->nrows;
    C.m = M->ncols;
    C.ptr.assign(M->rowptr, M->rowptr + M->nrows + 1);
    for (int i = 0; i < C.n; ++i)
        if (C.ptr[i + 1] < C.ptr[i]) throw ApiError(AMGMPCG_INVALID_ARG, std::string(what) + ": decreasing row pointers");
    C.col.assign(M->colind, M->colind + M->nnz);
    C.val.assign(M->val, M->val + M->nnz);
    for (int c : C.col)
        if (c < 0 || c >= C.m) throw ApiError(AMGMPCG_INVALID_ARG, std::string(what) + ": column index out of range");
    for (double v : C.val)
        if (!std::isfinite(v)) throw ApiError(AMGMPCG_NONFINITE, std::string(what) + ": non-finite value");
    return C;
}

int amgmpcg_setup_csr(const amgmpcg_csr* A, const amgmpcg_hierarchy* H, const amgmpcg_options* opts, void* stream,
                      amgmpcg_handle** out) {
    return guarded([&]() -> int {
        if (!out) throw ApiError(AMGMPCG_INVALID_ARG, "out pointer is NULL");
        *out = nullptr;
        validate_options(opts);
        if (opts->method != AMGMPCG_METHOD_MPCG) throw ApiError(AMGMPCG_INVALID_ARG, "CSR handles use the MPCG method");
        if (!H) throw ApiError(AMGMPCG_INVALID_ARG, "hierarchy is NULL");
        if (H->nlevels < 1 || H->nlevels > amg::kMaxNB) throw ApiError(AMGMPCG_INVALID_ARG, "nlevels must be in 1..8");
        if (H->nlevels > 1 && !H->P) throw ApiError(AMGMPCG_INVALID_ARG, "prolongations are NULL");
        if (!(H->restrict_scale > 0.0) || !std::isfinite(H->restrict_scale))
            throw ApiError(AMGMPCG_INVALID_ARG, "restrict_scale must be finite and > 0");
        amg::host::Csr Ah = csr_copy(A, "A");
        if (Ah.n != Ah.m) throw ApiError(AMGMPCG_INVALID_ARG, "A must be square");
        if (!amg::host::csr_symmetric(Ah, 1e-12)) throw ApiError(AMGMPCG_NOT_SPD, "A is not symmetric");
        std::vector<amg::host::Csr> Ps(H->nlevels - 1);
        int rows = Ah.n;
        for (int l = H->nlevels - 2; l >= 0; --l) {
            Ps[l] = csr_copy(&H->P[l], "P");
            if (Ps[l].n != rows) throw ApiError(AMGMPCG_INVALID_ARG, "P[l] rows must equal the unknowns of level l+1");
            rows = Ps[l].m;
        }
        const auto t0 = std::chrono::steady_clock::now();
        auto h = std::make_unique<amgmpcg_handle>();
        const int64_t bytes0 = amg::g_devbuf_bytes;
        hipStream_t s = (hipStream_t)stream;
        h->s.reset(amg::new_csr_solver(opts->precision, Ah, Ps, H->restrict_scale, *opts, s));
        h->bytes = amg::g_devbuf_bytes - bytes0;
        h->setup_ms = ms_since(t0);
        *out = h.release();
        return AMGMPCG_OK;
    });
}

int amgmpcg_setup_stencil(const amgmpcg_grid* grid, const double* stencil, const amgmpcg_options* opts,
                          void* stream, amgmpcg_handle** out) {
    return guarded([&]() -> int {
        if (!out) throw ApiError(AMGMPCG_INVALID_ARG, "out pointer is NULL");
        *out = nullptr;
        validate_grid(grid);
        validate_options(opts);
        if (grid->dim != 2) throw ApiError(AMGMPCG_INVALID_ARG, "the 9-point finest stencil needs dim = 2");
        if (grid->kappa) throw ApiError(AMGMPCG_INVALID_ARG, "kappa must be NULL with a finest stencil");
        if (!stencil) throw ApiError(AMGMPCG_INVALID_ARG, "stencil is NULL");
        for (int q = 0; q < 9; ++q) {
            if (!std::isfinite(stencil[q])) throw ApiError(AMGMPCG_NONFINITE, "non-finite stencil");
            if (stencil[q] != stencil[8 - q]) throw ApiError(AMGMPCG_INVALID_ARG, "the stencil must be symmetric");
        }
        if (!(stencil[4] > 0.0)) throw ApiError(AMGMPCG_NOT_SPD, "non-positive stencil centre");
        const auto t0 = std::chrono::steady_clock::now();
        auto h = std::make_unique<amgmpcg_handle>();
        const int64_t bytes0 = amg::g_devbuf_bytes;
        hipStream_t s = (hipStream_t)stream;
        h->s.reset(amg::new_grid_solver(opts->precision, 2, *grid, *opts, s, stencil));
        h->bytes = amg::g_devbuf_bytes - bytes0;
        h->setup_ms = ms_since(t0);
        *out = h.release();
        return AMGMPCG_OK;
    });
}

int amgmpcg_solve(amgmpcg_handle* h, const double* b_dev, double* x_dev, double tol, int32_t maxit,
                  amgmpcg_info* info) {
    return guarded([&]() -> int {
        if (!h || !h->s) throw ApiError(AMGMPCG_INVALID_ARG, "handle is NULL");
        if (!b_dev || !x_dev) throw ApiError(AMGMPCG_INVALID_ARG, "b or x is NULL");
        if (!(tol >= 0.0) || !std::isfinite(tol)) throw ApiError(AMGMPCG_INVALID_ARG, "tol must be finite and >= 0");
        const int st = h->s->solve(b_dev, x_dev, tol, maxit, info);
        if (info) info->setup_ms = h->setup_ms;
        return st;
    });
}

int amgmpcg_solve_host(amgmpcg_handle* h, const double* b, double* x, double tol, int32_t maxit,
                       amgmpcg_info* info) {
    return guarded([&]() -> int {
        if (!h || !h->s) throw ApiError(AMGMPCG_INVALID_ARG, "handle is NULL");
        if (!b || !x) throw ApiError(AMGMPCG_INVALID_ARG, "b or x is NULL");
        int n = h->s->n_axis.back();
        size_t N = (size_t)std::llround(std::pow((double)n, h->s->dim));
        double *db = nullptr, *dx = nullptr;
        HIPCHK(hipMalloc((void**)&db, N * sizeof(double)));
        hipError_t e = hipMalloc((void**)&dx, N * sizeof(double));
        if (e != hipSuccess) {
            (void)hipFree(db);
            HIPCHK(e);
        }
        int st;
        try {
            HIPCHK(hipMemcpy(db, b, N * sizeof(double), hipMemcpyHostToDevice));
            HIPCHK(hipMemcpy(dx, x, N * sizeof(double), hipMemcpyHostToDevice));
            st = h->s->solve(db, dx, tol, maxit, info);
            if (info) info->setup_ms = h->setup_ms;
            HIPCHK(hipMemcpy(x, dx, N * sizeof(double), hipMemcpyDeviceToHost));
        } catch (...) {
            (void)hipFree(db);
            (void)hipFree(dx);
            throw;
        }
        (void)hipFree(db);
        (void)hipFree(dx);
        return st;
    });
}

int amgmpcg_mg_block(amgmpcg_handle* h, const double* r_dev, double* Z_dev) {
    return guarded([&]() -> int {
        if (!h || !h->s) throw ApiError(AMGMPCG_INVALID_ARG, "handle is NULL");
        if (!r_dev || !Z_dev) throw ApiError(AMGMPCG_INVALID_ARG, "r or Z is NULL");
        h->s->mg_block(r_dev, Z_dev);
        return AMGMPCG_OK;
    });
}

int amgmpcg_level_count(const amgmpcg_handle* h, int32_t* nlevels, int32_t* nb) {
    return guarded([&]() -> int {
        if (!h || !h->s) throw ApiError(AMGMPCG_INVALID_ARG, "handle is NULL");
        if (nlevels) *nlevels = h->s->nlev;
        if (nb) *nb = h->s->nb;
        return AMGMPCG_OK;
    });
}

int amgmpcg_level_size(const amgmpcg_handle* h, int32_t level, int32_t* n_axis) {
    return guarded([&]() -> int {
        if (!h || !h->s || !n_axis) throw ApiError(AMGMPCG_INVALID_ARG, "NULL argument");
        if (level < 0 || level >= h->s->nlev) throw ApiError(AMGMPCG_INVALID_ARG, "level out of range");
        *n_axis = h->s->n_axis[level];
        return AMGMPCG_OK;
    });
}

int amgmpcg_level_stencil(const amgmpcg_handle* h, int32_t level, double* out) {
    return guarded([&]() -> int {
        if (!h || !h->s || !out) throw ApiError(AMGMPCG_INVALID_ARG, "NULL argument");
        h->s->level_stencil(level, out);
        return AMGMPCG_OK;
    });
}

int amgmpcg_history(const amgmpcg_handle* h, int32_t cap, double* alpha_out, double* resnorm_out, int32_t* count) {
    return guarded([&]() -> int {
        if (!h || !h->s) throw ApiError(AMGMPCG_INVALID_ARG, "handle is NULL");
        if (cap < 0) throw ApiError(AMGMPCG_INVALID_ARG, "cap must be >= 0");
        int c = 0;
        h->s->history(cap, alpha_out, resnorm_out, &c);
        if (count) *count = c;
        return AMGMPCG_OK;
    });
}

int amgmpcg_time_kernels(amgmpcg_handle* h, int32_t reps, double* ms_out, int32_t cap, int32_t* count) {
    return guarded([&]() -> int {
        if (!h || !h->s || !ms_out) throw ApiError(AMGMPCG_INVALID_ARG, "NULL argument");
        if (reps < 1 || cap < 0) throw ApiError(AMGMPCG_INVALID_ARG, "reps must be >= 1");
        const int c = h->s->time_kernels(reps, ms_out, cap);
        if (count) *count = c;
        return AMGMPCG_OK;
    });
}

int amgmpcg_profile_solve(amgmpcg_handle* h, const double* b_dev, double* x_dev, double tol, int32_t maxit,
                          amgmpcg_info* info, double* ms_out, int32_t cap, int32_t* count, int32_t* samples) {
    return guarded([&]() -> int {
        if (!h || !h->s) throw ApiError(AMGMPCG_INVALID_ARG, "handle is NULL");
        if (!b_dev || !x_dev || !ms_out) throw ApiError(AMGMPCG_INVALID_ARG, "NULL argument");
        if (!(tol >= 0.0) || !std::isfinite(tol)) throw ApiError(AMGMPCG_INVALID_ARG, "tol must be finite and >= 0");
        if (cap < 0) throw ApiError(AMGMPCG_INVALID_ARG, "cap must be >= 0");
        amgmpcg_info local{};
        int smp = 0;
        const int c = h->s->profile_solve(b_dev, x_dev, tol, maxit, &local, ms_out, cap, &smp);
        local.setup_ms = h->setup_ms;
        if (info) *info = local;
        if (count) *count = c;
        if (samples) *samples = smp;
        return local.status;
    });
}

int amgmpcg_setup_batched(int32_t count, const amgmpcg_grid* grids, const amgmpcg_options* opts, void* stream,
                          amgmpcg_handle** out) {
    return guarded([&]() -> int {
        if (!out) throw ApiError(AMGMPCG_INVALID_ARG, "out pointer is NULL");
        *out = nullptr;
        if (count < 1 || !grids) throw ApiError(AMGMPCG_INVALID_ARG, "need count >= 1 problems");
        validate_options(opts);
        if (opts->nu > 2) throw ApiError(AMGMPCG_INVALID_ARG, "batched solves support nu = 1 or 2");
        const int dim = grids[0].dim;
        for (int i = 0; i < count; ++i) {
            validate_grid(&grids[i]);
            if (grids[i].dim != dim) throw ApiError(AMGMPCG_INVALID_ARG, "all batched problems need the same dim");
            if (grids[i].kappa) throw ApiError(AMGMPCG_INVALID_ARG, "batched problems are Poisson (kappa must be NULL)");
            if (grids[i].nlevels > 6) throw ApiError(AMGMPCG_INVALID_ARG, "batched problems support up to 6 levels");
        }
        if (opts->m != 1 || opts->method != AMGMPCG_METHOD_MPCG)
            throw ApiError(AMGMPCG_INVALID_ARG, "batched solves use the MPCG method with m = 1");
        const auto t0 = std::chrono::steady_clock::now();
        auto h = std::make_unique<amgmpcg_handle>();
        const int64_t bytes0 = amg::g_devbuf_bytes;
        hipStream_t s = (hipStream_t)stream;
        h->bs.reset(amg::new_batched_solver(opts->precision, dim, count, grids, *opts, s));
        h->bytes = amg::g_devbuf_bytes - bytes0;
        h->setup_ms = ms_since(t0);
        *out = h.release();
        return AMGMPCG_OK;
    });
}

int amgmpcg_solve_batched(amgmpcg_handle* h, const double* b_dev, double* x_dev, double tol, int32_t maxit,
                          amgmpcg_info* infos, double* batch_ms) {
    return guarded([&]() -> int {
        if (!h || !h->bs) throw ApiError(AMGMPCG_INVALID_ARG, "handle is not a batched handle");
        if (!b_dev || !x_dev) throw ApiError(AMGMPCG_INVALID_ARG, "b or x is NULL");
        if (!(tol >= 0.0) || !std::isfinite(tol)) throw ApiError(AMGMPCG_INVALID_ARG, "tol must be finite and >= 0");
        const int st = h->bs->solve(b_dev, x_dev, tol, maxit, infos, batch_ms);
        if (infos)
            for (int i = 0; i < h->bs->count; ++i) {
                infos[i].relres_true = -1.0;
                infos[i].setup_ms = h->setup_ms;
            }
        return st;
    });
}

int amgmpcg_workspace_bytes(const amgmpcg_handle* h, int64_t* bytes) {
    return guarded([&]() -> int {
        if (!h || (!h->s && !h->bs)) throw ApiError(AMGMPCG_INVALID_ARG, "handle is NULL");
        if (!bytes) throw ApiError(AMGMPCG_INVALID_ARG, "bytes is NULL");
        *bytes = h->s ? h->s->workspace_need() : h->bytes;
        return AMGMPCG_OK;
    });
}

int amgmpcg_bind_workspace(amgmpcg_handle* h, void* device_ptr, int64_t bytes) {
    return guarded([&]() -> int {
        if (!h || (!h->s && !h->bs)) throw ApiError(AMGMPCG_INVALID_ARG, "handle is NULL");
        if (!h->s) throw ApiError(AMGMPCG_INVALID_ARG, "a batched handle owns its memory");
        if (!device_ptr) throw ApiError(AMGMPCG_INVALID_ARG, "workspace pointer is NULL");
        if (reinterpret_cast<uintptr_t>(device_ptr) % amg::kWsAlign != 0)
            throw ApiError(AMGMPCG_INVALID_ARG, "workspace must be 256-byte aligned");
        const int64_t need = h->s->workspace_need();
        if (bytes < need)
            throw ApiError(AMGMPCG_INVALID_ARG,
                           "workspace too small: " + std::to_string(bytes) + " < " + std::to_string(need) + " bytes");
        hipPointerAttribute_t attr;
        if (hipPointerGetAttributes(&attr, device_ptr) != hipSuccess || attr.type != hipMemoryTypeDevice) {
            (void)hipGetLastError();
            throw ApiError(AMGMPCG_INVALID_ARG, "workspace is not device memory");
        }
        h->s->bind_workspace(static_cast<char*>(device_ptr), bytes);
        return AMGMPCG_OK;
    });
}

int amgmpcg_batched_size(const amgmpcg_handle* h, int32_t* count, int64_t* total_dofs) {
    return guarded([&]() -> int {
        if (!h || !h->bs) throw ApiError(AMGMPCG_INVALID_ARG, "handle is not a batched handle");
        if (count) *count = h->bs->count;
        if (total_dofs) *total_dofs = h->bs->total;
        return AMGMPCG_OK;
    });
}

int amgmpcg_gram_pinv(const double* G, int32_t nb, double tau, double* Gplus, int32_t* rank) {
    return guarded([&]() -> int {
        if (!G || !Gplus || !rank) throw ApiError(AMGMPCG_INVALID_ARG, "NULL argument");
        if (nb < 1 || nb > amg::kMaxNB) throw ApiError(AMGMPCG_INVALID_ARG, "nb must be in 1..8");
        if (!(tau > 0.0)) throw ApiError(AMGMPCG_INVALID_ARG, "tau must be > 0");
        amg::DevBuf<double> d;
        d.alloc(2 * (size_t)nb * nb + 1);
        HIPCHK(hipMemcpy(d.p, G, sizeof(double) * nb * nb, hipMemcpyHostToDevice));
        int* drank = (int*)(d.p + 2 * nb * nb);
        double* dGp = d.p + nb * nb;
        amg::launch_pinv(nb, d.p, tau, dGp, drank);
        HIPCHK(hipMemcpy(Gplus, dGp, sizeof(double) * nb * nb, hipMemcpyDeviceToHost));
        int r = 0;
        HIPCHK(hipMemcpy(&r, drank, sizeof(int), hipMemcpyDeviceToHost));
        *rank = r;
        return AMGMPCG_OK;
    });
}

int amgmpcg_gram_pinv_noalloc(const double* G, int32_t nb, double tau, double* Gplus, int32_t* rank) {
    return guarded([&]() -> int {
        if (!G || !Gplus || !rank) throw ApiError(AMGMPCG_INVALID_ARG, "NULL argument");
        if (nb < 1 || nb > amg::kMaxNB)
            throw ApiError(AMGMPCG_INVALID_ARG, "nb must be in 1..8 (the static staging holds an 8 x 8 Gram)");
        if (!(tau > 0.0)) throw ApiError(AMGMPCG_INVALID_ARG, "tau must be > 0");
        double* sc = amg::pinv_scratch();
        double* dG = sc;
        double* dGp = sc + amg::kMaxNB * amg::kMaxNB;
        int* drank = reinterpret_cast<int*>(sc + 2 * amg::kMaxNB * amg::kMaxNB);
        HIPCHK(hipMemcpy(dG, G, sizeof(double) * nb * nb, hipMemcpyHostToDevice));
        amg::launch_pinv(nb, dG, tau, dGp, drank);
        HIPCHK(hipMemcpy(Gplus, dGp, sizeof(double) * nb * nb, hipMemcpyDeviceToHost));
        int r = 0;
        HIPCHK(hipMemcpy(&r, drank, sizeof(int), hipMemcpyDeviceToHost));
        *rank = r;
        return AMGMPCG_OK;
    });
}

int amgmpcg_residual(amgmpcg_handle* h, const double* b_dev, const double* x_dev, double* r_dev) {
    return guarded([&]() -> int {
        if (!h || !h->s) throw ApiError(AMGMPCG_INVALID_ARG, "handle is NULL");
        if (!b_dev || !x_dev || !r_dev) throw ApiError(AMGMPCG_INVALID_ARG, "NULL vector");
        if (r_dev == b_dev || r_dev == x_dev) throw ApiError(AMGMPCG_INVALID_ARG, "r may not alias b or x");
        h->s->residual(b_dev, x_dev, r_dev);
        return AMGMPCG_OK;
    });
}

int64_t amgmpcg_cnn_weight_count(void) { return amg::cnn::total_weights(); }

static void check_net(const amgmpcg_cnn* net) {
    if (!net) throw ApiError(AMGMPCG_INVALID_ARG, "network is NULL");
}

static void check_count(int64_t count) {
    if (count != amg::cnn::total_weights()) throw ApiError(AMGMPCG_INVALID_ARG, "weight count mismatch");
}

int amgmpcg_cnn_create(int32_t n, uint64_t seed, void* stream, amgmpcg_cnn** out) {
    return guarded([&]() -> int {
        if (!out) throw ApiError(AMGMPCG_INVALID_ARG, "out pointer is NULL");
        *out = nullptr;
        if (n < 1 || n > 1000) throw ApiError(AMGMPCG_INVALID_ARG, "n must be in 1..1000");
        auto c = std::make_unique<amgmpcg_cnn>();
        HIPCHK(c->net.init(n, seed, (hipStream_t)stream));
        *out = c.release();
        return AMGMPCG_OK;
    });
}

int amgmpcg_cnn_set_weights(amgmpcg_cnn* net, const float* w, int64_t count) {
    return guarded([&]() -> int {
        check_net(net);
        check_count(count);
        if (!w) throw ApiError(AMGMPCG_INVALID_ARG, "weights are NULL");
        HIPCHK(net->net.set_weights(w));
        return AMGMPCG_OK;
    });
}

int amgmpcg_cnn_get_weights(amgmpcg_cnn* net, float* w, int64_t count) {
    return guarded([&]() -> int {
        check_net(net);
        check_count(count);
        if (!w) throw ApiError(AMGMPCG_INVALID_ARG, "output is NULL");
        HIPCHK(net->net.get(net->net.w.p, w));
        return AMGMPCG_OK;
    });
}

int amgmpcg_cnn_get_gradients(amgmpcg_cnn* net, float* g, int64_t count) {
    return guarded([&]() -> int {
        check_net(net);
        check_count(count);
        if (!g) throw ApiError(AMGMPCG_INVALID_ARG, "output is NULL");
        HIPCHK(net->net.get(net->net.g.p, g));
        return AMGMPCG_OK;
    });
}

int amgmpcg_cnn_forward(amgmpcg_cnn* net, const double* r_dev, const uint16_t* lk_dev, double* d_dev) {
    return guarded([&]() -> int {
        check_net(net);
        if (!r_dev || !d_dev) throw ApiError(AMGMPCG_INVALID_ARG, "r or d is NULL");
        bool finite = true;
        HIPCHK(net->net.infer(r_dev, lk_dev, d_dev, &finite));
        return finite ? AMGMPCG_OK : AMGMPCG_NONFINITE;
    });
}

int amgmpcg_cnn_gradients(amgmpcg_cnn* net, const double* r_dev, const uint16_t* lk_dev, const double* e_dev,
                          double* loss) {
    return guarded([&]() -> int {
        check_net(net);
        if (!r_dev || !e_dev) throw ApiError(AMGMPCG_INVALID_ARG, "r or e is NULL");
        HIPCHK(net->net.step_pair(r_dev, lk_dev, e_dev, 0.f, loss));
        return AMGMPCG_OK;
    });
}

int amgmpcg_cnn_train_step(amgmpcg_cnn* net, const double* r_dev, const uint16_t* lk_dev, const double* e_dev,
                           float lr, double* loss) {
    return guarded([&]() -> int {
        check_net(net);
        if (!r_dev || !e_dev) throw ApiError(AMGMPCG_INVALID_ARG, "r or e is NULL");
        if (!(lr > 0.f) || !std::isfinite(lr)) throw ApiError(AMGMPCG_INVALID_ARG, "lr must be finite and > 0");
        HIPCHK(net->net.step_pair(r_dev, lk_dev, e_dev, lr, loss));
        return AMGMPCG_OK;
    });
}

int amgmpcg_cnn_energy_step(amgmpcg_cnn* net, amgmpcg_handle* h, const double* r_dev, const uint16_t* lk_dev,
                            const double* e_dev, int32_t marginal, float lr, double* loss) {
    return guarded([&]() -> int {
        check_net(net);
        if (!h || !h->s) throw ApiError(AMGMPCG_INVALID_ARG, "handle is NULL");
        if (!r_dev || !e_dev) throw ApiError(AMGMPCG_INVALID_ARG, "r or e is NULL");
        if (!(lr >= 0.f) || !std::isfinite(lr)) throw ApiError(AMGMPCG_INVALID_ARG, "lr must be finite and >= 0");
        if (h->s->dim != 3 || h->s->n_axis.back() != net->net.n)
            throw ApiError(AMGMPCG_DIM_MISMATCH, "the handle's grid differs from the network's");
        if (marginal != 0 && marginal != 1) throw ApiError(AMGMPCG_INVALID_ARG, "marginal must be 0 or 1");
        amg::cnn::Net& N = net->net;
        N.forward(nullptr, r_dev, lk_dev, N.stream, true);
        N.output_vector(N.stream);
        h->s->apply_fine(N.dvec.p, N.qvec.p, N.stream);
        if (marginal) {
            h->s->project_prepare(r_dev, N.rvec.p, N.stream);
            h->s->project_direction(N.dvec.p, N.qvec.p, N.q2vec.p, N.stream);
            N.loss_energy(N.rvec.p, N.q2vec.p, e_dev, N.stream);
        } else {
            N.loss_energy(r_dev, N.qvec.p, e_dev, N.stream);
        }
        N.backward(N.stream);
        if (lr > 0.f) N.adam(lr, N.stream);
        HIPCHK(N.read_loss(loss));
        return AMGMPCG_OK;
    });
}

int amgmpcg_energy_grad(amgmpcg_handle* h, const double* d_dev, const double* r_dev, const double* e_dev,
                        int32_t marginal, double* grad_dev, double* loss) {
    return guarded([&]() -> int {
        if (!h || !h->s) throw ApiError(AMGMPCG_INVALID_ARG, "handle is NULL");
        if (!d_dev || !r_dev || !e_dev || !grad_dev) throw ApiError(AMGMPCG_INVALID_ARG, "NULL vector");
        if (marginal != 0 && marginal != 1) throw ApiError(AMGMPCG_INVALID_ARG, "marginal must be 0 or 1");
        amg::SolverBase& S = *h->s;
        const int n = S.n_axis.back();
        const int N = (int)std::llround(std::pow((double)n, S.dim));
        amg::DevBuf<double> q, qh, rh, part, sc;
        q.alloc(N);
        part.alloc((size_t)3 * amg::cnn::kSumBlocks);
        sc.alloc(4);
        hipStream_t st = nullptr;
        S.apply_fine(d_dev, q.p, st);
        const double* rr = r_dev;
        const double* qq = q.p;
        if (marginal) {
            qh.alloc(N);
            rh.alloc(N);
            S.project_prepare(r_dev, rh.p, st);
            S.project_direction(d_dev, q.p, qh.p, st);
            rr = rh.p;
            qq = qh.p;
        }
        amg::cnn::k_dots3<<<amg::cnn::kSumBlocks, amg::cnn::kCB, 0, st>>>(d_dev, qq, rr, e_dev, N, part.p);
        amg::cnn::k_energy_finish<<<1, amg::kRedBlock, 0, st>>>(part.p, amg::cnn::kSumBlocks, sc.p);
        amg::cnn::k_energy_grad64<<<(N + amg::cnn::kCB - 1) / amg::cnn::kCB, amg::cnn::kCB, 0, st>>>(sc.p, qq, rr,
                                                                                                  grad_dev, N);
        HIPCHK(hipGetLastError());
        double hs[4];
        HIPCHK(hipMemcpyAsync(hs, sc.p, sizeof(hs), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (loss) *loss = hs[3];
        return AMGMPCG_OK;
    });
}

int amgmpcg_cnn_time_forward(amgmpcg_cnn* net, const double* r_dev, const uint16_t* lk_dev, int32_t reps,
                             double* ms) {
    return guarded([&]() -> int {
        check_net(net);
        if (!r_dev || !ms) throw ApiError(AMGMPCG_INVALID_ARG, "NULL argument");
        if (reps < 1) throw ApiError(AMGMPCG_INVALID_ARG, "reps must be >= 1");
        hipStream_t s = net->net.stream;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        HIPCHK(hipEventCreate(&e0));
        hipError_t err = hipEventCreate(&e1);
        if (err == hipSuccess) err = hipEventRecord(e0, s);
        for (int i = 0; i < reps && err == hipSuccess; ++i) net->net.forward(nullptr, r_dev, lk_dev, s);
        if (err == hipSuccess) err = hipGetLastError();
        if (err == hipSuccess) err = hipEventRecord(e1, s);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float t = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
        (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        HIPCHK(err);
        *ms = double(t) / reps;
        return AMGMPCG_OK;
    });
}

int amgmpcg_cnn_layer(amgmpcg_cnn* net, int32_t layer, int32_t op, int32_t S, const uint16_t* A_dev,
                      const uint16_t* B_dev, void* out_dev) {
    return guarded([&]() -> int {
        check_net(net);
        if (layer < 0 || layer > 10) throw ApiError(AMGMPCG_INVALID_ARG, "layer must be in 0..10");
        if (op < 0 || op > 2) throw ApiError(AMGMPCG_INVALID_ARG, "op must be 0, 1 or 2");
        if (S < 1 || S > 512) throw ApiError(AMGMPCG_INVALID_ARG, "S must be in 1..512");
        if (!A_dev || !out_dev || (op == 2 && !B_dev)) throw ApiError(AMGMPCG_INVALID_ARG, "NULL tensor");
        HIPCHK(net->net.layer_op(layer, op, S, A_dev, B_dev, out_dev));
        return AMGMPCG_OK;
    });
}

void amgmpcg_cnn_destroy(amgmpcg_cnn* net) { delete net; }

int amgmpcg_attach_cnn(amgmpcg_handle* h, amgmpcg_cnn* net) {
    return guarded([&]() -> int {
        if (!h || !h->s) throw ApiError(AMGMPCG_INVALID_ARG, "handle is NULL");
        const int64_t bytes0 = amg::g_devbuf_bytes;
        h->s->attach(net ? &net->net : nullptr);
        h->bytes += amg::g_devbuf_bytes - bytes0;
        return AMGMPCG_OK;
    });
}

int amgmpcg_log_kappa(amgmpcg_handle* h, uint16_t* lk_dev) {
    return guarded([&]() -> int {
        if (!h || !h->s) throw ApiError(AMGMPCG_INVALID_ARG, "handle is NULL");
        if (!lk_dev) throw ApiError(AMGMPCG_INVALID_ARG, "output is NULL");
        if (h->s->dim != 3) throw ApiError(AMGMPCG_INVALID_ARG, "the learned direction needs a 3D problem");
        h->s->log_kappa(lk_dev);
        return AMGMPCG_OK;
    });
}

int amgmpcg_make_pairs(amgmpcg_handle* h, const double* b_dev, const double* xs_dev, const int32_t* ks,
                       int32_t nk, double* R_dev, double* E_dev) {
    return guarded([&]() -> int {
        if (!h || !h->s) throw ApiError(AMGMPCG_INVALID_ARG, "handle is NULL");
        if (!b_dev || !xs_dev || !ks || !R_dev || !E_dev) throw ApiError(AMGMPCG_INVALID_ARG, "NULL argument");
        if (nk < 1) throw ApiError(AMGMPCG_INVALID_ARG, "nk must be >= 1");
        for (int i = 0; i < nk; ++i)
            if (ks[i] < 0) throw ApiError(AMGMPCG_INVALID_ARG, "iteration counts must be >= 0");
        h->s->make_pairs(b_dev, xs_dev, ks, nk, R_dev, E_dev);
        return AMGMPCG_OK;
    });
}

void amgmpcg_destroy(amgmpcg_handle* h) { delete h; }

const char* amgmpcg_status_string(int s) {
    switch (s) {
        case AMGMPCG_OK: return "converged";
        case AMGMPCG_MAXIT: return "iteration limit reached";
        case AMGMPCG_BREAKDOWN: return "breakdown: every search direction dropped";
        case AMGMPCG_INVALID_ARG: return "invalid argument";
        case AMGMPCG_NOT_SPD: return "operator not SPD (non-positive diagonal)";
        case AMGMPCG_DIM_MISMATCH: return "dimension mismatch";
        case AMGMPCG_NONFINITE: return "non-finite value";
        case AMGMPCG_OOM: return "out of memory";
        case AMGMPCG_HIP_ERROR: return "HIP runtime error";
        case AMGMPCG_UNAVAILABLE: return "entry point switched off in this build";
        default: return "unknown status";
    }
}

const char* amgmpcg_last_error(void) { return amg::g_last_error.c_str(); }

}  // extern "C"

