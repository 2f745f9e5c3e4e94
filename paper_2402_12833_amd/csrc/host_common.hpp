// Host-side definitions shared by the translation units of libamgmpcg:
// errors, device buffers, the solver interfaces the C entry points call, and
// the factories of the solver types (each instantiated in its own unit).
#pragma once
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "amgmpcg.h"
#include "common.hpp"
#include "grid_kernels.hpp"
#include "setup.hpp"
#include "small_kernels.hpp"

namespace amg {

namespace cnn {
class Net;
}


static_assert(kOK == AMGMPCG_OK && kMAXIT == AMGMPCG_MAXIT && kBREAKDOWN == AMGMPCG_BREAKDOWN &&
                  kNONFINITE == AMGMPCG_NONFINITE,
              "status codes");

extern thread_local std::string g_last_error;

struct ApiError : std::runtime_error {
    int code;
    ApiError(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPCHK(expr)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) {                                                                        \
            if (e_ == hipErrorOutOfMemory)                                                             \
                throw ApiError(AMGMPCG_OOM, std::string("out of device memory: ") + #expr);            \
            throw ApiError(AMGMPCG_HIP_ERROR,                                                          \
                           std::string(hipGetErrorString(e_)) + " at " + #expr + " line " +            \
                               std::to_string(__LINE__));                                              \
        }                                                                                              \
    } while (0)

// Launch kernel k with the dispatch's own start and end times recorded on
// e0 and e1 (hipExtLaunchKernel), so hipEventElapsedTime(e0, e1) is the
// kernel's duration without the launch latency around it.  Each argument is
// converted to the kernel's parameter type first.
template <typename... P, typename... A>
void launch_with_events(void (*k)(P...), dim3 grid, dim3 block, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                        A&&... a) {
    std::tuple<P...> t{std::forward<A>(a)...};
    void* args[sizeof...(P)];
    std::apply([&](auto&... v) {
        int i = 0;
        ((args[i++] = static_cast<void*>(&v)), ...);
    }, t);
    HIPCHK(hipExtLaunchKernel(reinterpret_cast<const void*>(k), grid, block, args, 0, s, e0, e1, 0));
}

#ifndef AMG_FINE_BLOCKS
#define AMG_FINE_BLOCKS 2048
#endif
constexpr int kMaxFineBlocks = AMG_FINE_BLOCKS;   // blocks of the fine-level kernels (multiple of 8)
constexpr int kTailMax = 4096;          // prolongation outputs up to this size: single-block chain
constexpr int kRestrictTailMax = 512;   // restriction outputs up to this size: single-block chain
constexpr int kProlong2Max = 65536;     // two carry steps in one launch up to this many target nodes
constexpr int kPartRow = 2 + 1 + kMaxNB * kMaxNB + (kMaxNB * (kMaxNB + 1) / 2 + kMaxNB) + 1;

// Device bytes held by the DevBufs of this thread (a handle's footprint is
// the difference across its construction).
extern thread_local int64_t g_devbuf_bytes;

template <typename T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    bool ext = false;   // p lies in a caller's workspace (amgmpcg_bind_workspace): not freed here
    void alloc(size_t count) {
        free();
        if (count == 0) return;
        HIPCHK(hipMalloc((void**)&p, count * sizeof(T)));
        n = count;
        g_devbuf_bytes += (int64_t)(count * sizeof(T));
    }
    void free() {
        if (p && !ext) {
            (void)hipFree(p);
            g_devbuf_bytes -= (int64_t)(n * sizeof(T));
        }
        p = nullptr;
        n = 0;
        ext = false;
    }
    ~DevBuf() { free(); }
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n), ext(o.ext) {
        o.p = nullptr;
        o.n = 0;
        o.ext = false;
    }
    DevBuf& operator=(DevBuf&& o) noexcept {
        if (this != &o) {
            free();
            p = o.p;
            n = o.n;
            ext = o.ext;
            o.p = nullptr;
            o.n = 0;
            o.ext = false;
        }
        return *this;
    }
};

// A device buffer of a handle, type-erased: where its pointer lives, its size
// and whether it lies in a caller's workspace.
struct BufRef {
    void** p;
    size_t bytes;
    bool* ext;
};
template <typename T>
BufRef buf_ref(DevBuf<T>& b) {
    return BufRef{reinterpret_cast<void**>(&b.p), b.n * sizeof(T), &b.ext};
}

// Alignment of every buffer placed in a caller's workspace.
constexpr size_t kWsAlign = 256;
inline size_t ws_round(size_t bytes) { return (bytes + kWsAlign - 1) / kWsAlign * kWsAlign; }

class SolverBase {
   public:
    virtual ~SolverBase() = default;
    virtual int solve(const double* b_dev, double* x_dev, double tol, int maxit, amgmpcg_info* info) = 0;
    virtual void mg_block(const double* r_dev, double* Z_dev) = 0;
    virtual void level_stencil(int level, double* out) = 0;
    virtual void history(int cap, double* alpha, double* res, int* count) = 0;
    virtual int time_kernels(int reps, double* ms, int cap) = 0;
    virtual int profile_solve(const double* b_dev, double* x_dev, double tol, int maxit, amgmpcg_info* info,
                              double* ms, int cap, int* samples) = 0;
    virtual void attach(cnn::Net* net) = 0;
    virtual void residual(const double* b_dev, const double* x_dev, double* r_dev) = 0;
    virtual void make_pairs(const double* b_dev, const double* xs_dev, const int* ks, int nk, double* R_dev,
                            double* E_dev) = 0;
    virtual void log_kappa(unsigned short* lk_dev) = 0;
    virtual void apply_fine(const double* x_dev, double* y_dev, hipStream_t s) = 0;
    virtual void project_prepare(const double* r_dev, double* rhat_dev, hipStream_t s) = 0;
    virtual void project_direction(const double* d_dev, const double* q_dev, double* qhat_dev, hipStream_t s) = 0;
    // Every device buffer of the handle (not the control words), and what
    // to redo once they have moved: pointers cached in operator structs,
    // the captured iteration graph (its kernel arguments hold the old
    // addresses).
    virtual void buffers(std::vector<BufRef>& out) = 0;
    virtual void rebound() = 0;
    virtual hipStream_t stream() const = 0;

    // Bytes of a caller workspace that holds all buffers, each at a
    // kWsAlign-aligned offset.
    int64_t workspace_need() {
        std::vector<BufRef> v;
        buffers(v);
        int64_t s = 0;
        for (const BufRef& b : v) s += (int64_t)ws_round(b.bytes);
        return s;
    }

    // Move every buffer into [ws, ws + bytes) (contents copied on the
    // handle's stream), free the handle's own copies and redo what holds
    // the old addresses.  The caller checks size and alignment first.
    void bind_workspace(char* ws, int64_t bytes) {
        std::vector<BufRef> v;
        buffers(v);
        std::vector<std::pair<void*, size_t>> old;
        size_t off = 0;
        for (const BufRef& b : v) {
            if (b.bytes == 0 || !*b.p) continue;
            char* dst = ws + off;
            if ((int64_t)(off + b.bytes) > bytes) throw ApiError(AMGMPCG_INVALID_ARG, "workspace too small");
            HIPCHK(hipMemcpyAsync(dst, *b.p, b.bytes, hipMemcpyDeviceToDevice, stream()));
            if (!*b.ext) old.emplace_back(*b.p, b.bytes);
            *b.p = dst;
            *b.ext = true;
            off += ws_round(b.bytes);
        }
        HIPCHK(hipStreamSynchronize(stream()));
        for (auto& o : old) {
            (void)hipFree(o.first);
            g_devbuf_bytes -= (int64_t)o.second;
        }
        rebound();
    }

    bool bound() {
        std::vector<BufRef> v;
        buffers(v);
        for (const BufRef& b : v)
            if (*b.ext) return true;
        return false;
    }

    cnn::Net* net_ = nullptr;
    int dim = 0, nlev = 0, nb = 0;
    std::vector<int> n_axis;   // per level, 0 = coarsest
};

static int fine_blocks(int N, int cap = kMaxFineBlocks) {
    int b = (N + kBlock - 1) / kBlock;
    if (b > cap) b = cap;
    if (b >= kNumXcd) b = (b / kNumXcd) * kNumXcd;
    return b < 1 ? 1 : b;
}

// The block SpMM + Gram and W = Q^T Z kernels carry 27-44 accumulators per
// thread: fewer, longer-running blocks amortise their block reductions.
#ifndef AMG_GRAM_BLOCKS
#define AMG_GRAM_BLOCKS 1024
#endif
constexpr int kGramBlocks = AMG_GRAM_BLOCKS;

// z-marching SpMM + Gram on 3D grids: TY rows per tile (a multiple of 2) and
// kz planes per unit.
#ifndef AMG_ZTILE_TY
#define AMG_ZTILE_TY 2
#endif
#ifndef AMG_ZTILE_KZ
#define AMG_ZTILE_KZ 0
#endif
constexpr int kZTY = AMG_ZTILE_TY;
constexpr int kZKZ = AMG_ZTILE_KZ;    // 0: split z so that the units fill the resident blocks once
constexpr int kNumCU = 256;
constexpr int kGramRow = kMaxNB * (kMaxNB + 1) / 2 + kMaxNB;   // Gram + P^T r partial values
constexpr size_t kBlockSlack = 16;   // elements past the last slot (16-byte chunk reads)

// Elements per direction-block slot: b columns (even stride) per node, rounded
// up to 64 elements so that every slot starts 256-byte aligned.
inline size_t slot_elems(int nb, int N) { return ((size_t)even_up(nb) * N + 63) / 64 * 64; }


class BatchedBase {
   public:
    virtual ~BatchedBase() = default;
    virtual int solve(const double* b_dev, double* x_dev, double tol, int maxit, amgmpcg_info* infos,
                      double* batch_ms) = 0;
    int count = 0;
    int64_t total = 0;
};

// Factories, one translation unit per solver type and precision.
SolverBase* new_grid_solver(int precision, int dim, const amgmpcg_grid& g, const amgmpcg_options& o,
                            hipStream_t stream, const double* st9);
SolverBase* new_csr_solver(int precision, const host::Csr& A, const std::vector<host::Csr>& Ps, double rscale,
                           const amgmpcg_options& o, hipStream_t stream);
BatchedBase* new_batched_solver(int precision, int dim, int count, const amgmpcg_grid* grids,
                                const amgmpcg_options& o, hipStream_t stream);

}  // namespace amg
