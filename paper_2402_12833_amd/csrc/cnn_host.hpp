// Host driver of the U-Net (weights, activation buffers, launch sequences).
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cmath>
#include <cstdint>
#include <vector>

#include "cnn.hpp"

namespace amg {
namespace cnn {

struct LayerSpec {
    int taps, cin, cout;
};
// w1..w11 (input padded to 16 channels; output layer 1x1 with 16 padded outputs)
constexpr LayerSpec kLayers[11] = {{27, 16, 16}, {27, 16, 16}, {27, 16, 32}, {27, 32, 32}, {27, 32, 64}, {27, 64, 64},
                                   {27, 96, 32}, {27, 32, 32}, {27, 48, 16}, {27, 16, 16}, {1, 16, 16}};
constexpr int kInChannels = 2;
constexpr int kSumBlocks = 512;   // blocks of the dot-product partials
constexpr int kSqBlocks = 1024;   // blocks of the sum-of-squares partials (8 values per thread at 128^3)

inline int64_t layer_size(int l) { return (int64_t)kLayers[l].taps * kLayers[l].cout * kLayers[l].cin; }
inline int64_t total_weights() {
    int64_t s = 0;
    for (int l = 0; l < 11; ++l) s += layer_size(l);
    return s;
}

template <typename X>
struct Buf {
    X* p = nullptr;
    size_t n = 0;
    void alloc(size_t count, hipError_t& err) {
        if (err != hipSuccess) return;
        err = hipMalloc((void**)&p, count * sizeof(X));
        if (err == hipSuccess) n = count;
        else p = nullptr;
    }
    ~Buf() {
        if (p) (void)hipFree(p);
    }
};

class Net {
   public:
    int n = 0, S = 0;
    hipStream_t stream = nullptr;

    // returns hipSuccess or the first allocation error
    hipError_t init(int n_, uint64_t seed, hipStream_t s) {
        n = n_;
        S = (n + 3) / 4 * 4;
        stream = s;
        hipError_t err = hipSuccess;
        const size_t V0 = (size_t)S * S * S, V1 = V0 / 8, V2 = V1 / 8;
        x0.alloc(V0 * 16, err);
        e1.alloc(V0 * 16, err);
        e2.alloc(V0 * 16, err);
        p1.alloc(V1 * 16, err);
        e3.alloc(V1 * 32, err);
        e4.alloc(V1 * 32, err);
        p2.alloc(V2 * 32, err);
        b1.alloc(V2 * 64, err);
        b2.alloc(V2 * 64, err);
        c1.alloc(V1 * 96, err);
        d1.alloc(V1 * 32, err);
        d2.alloc(V1 * 32, err);
        c2.alloc(V0 * 48, err);
        d3.alloc(V0 * 16, err);
        d4.alloc(V0 * 16, err);
        out.alloc(V0, err);
        g0a.alloc(V0 * 16, err);
        g0b.alloc(V0 * 16, err);
        g0c.alloc(V0 * 48, err);
        g1a.alloc(V1 * 96, err);
        g1b.alloc(V1 * 32, err);
        g1c.alloc(V1 * 32, err);
        g2a.alloc(V2 * 64, err);
        g2b.alloc(V2 * 64, err);
        g2c.alloc(V2 * 32, err);
        small.alloc(16, err);
        dvec.alloc((size_t)n * n * n, err);
        qvec.alloc((size_t)n * n * n, err);
        rvec.alloc((size_t)n * n * n, err);
        q2vec.alloc((size_t)n * n * n, err);
        flag.alloc(1, err);
        // block partials: one per block of the loss kernel, or up to three
        // values (k_dots3) per block of the kSumBlocks-block reductions
        static_assert(kSqBlocks <= 3 * kSumBlocks, "partials buffer");
        part.alloc((V0 + kCB - 1) / kCB > 3 * kSumBlocks ? (V0 + kCB - 1) / kCB : 3 * kSumBlocks, err);
        const int64_t NW = total_weights();
        w.alloc(NW, err);
        m.alloc(NW, err);
        v.alloc(NW, err);
        g.alloc(NW, err);
        wb.alloc(NW, err);
        wt.alloc(NW, err);
        if (err != hipSuccess) return err;
        // He-normal initial weights on the host (splitmix64 + Box-Muller)
        std::vector<float> h(NW);
        uint64_t st = seed * 0x9E3779B97F4A7C15ull + 1;
        auto next = [&]() {
            uint64_t z = (st += 0x9E3779B97F4A7C15ull);
            z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
            z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
            return ((z ^ (z >> 31)) >> 11) * 0x1.0p-53;
        };
        int64_t off = 0;
        for (int l = 0; l < 11; ++l) {
            const LayerSpec L = kLayers[l];
            const int fan = L.taps * (l == 0 ? kInChannels : L.cin);
            const double sd = std::sqrt(2.0 / fan);
            for (int t = 0; t < L.taps; ++t)
                for (int co = 0; co < L.cout; ++co)
                    for (int ci = 0; ci < L.cin; ++ci) {
                        double u1 = next(), u2 = next();
                        if (u1 < 1e-300) u1 = 1e-300;
                        double val = sd * std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
                        if (l == 0 && ci >= kInChannels) val = 0.0;
                        if (l == 10 && co >= 1) val = 0.0;
                        h[off++] = (float)val;
                    }
        }
        return set_weights(h.data());
    }

    hipError_t set_weights(const float* host) {
        const int64_t NW = total_weights();
        hipError_t e = hipMemcpyAsync(w.p, host, NW * sizeof(float), hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = hipMemsetAsync(m.p, 0, NW * sizeof(float), stream);
        if (e == hipSuccess) e = hipMemsetAsync(v.p, 0, NW * sizeof(float), stream);
        if (e != hipSuccess) return e;
        step = 0;
        int64_t off = 0;
        for (int l = 0; l < 11; ++l) {
            const LayerSpec L = kLayers[l];
            const int cnt = (int)layer_size(l);
            k_weights_bf16<<<(cnt + kCB - 1) / kCB, kCB, 0, stream>>>(w.p + off, wb.p + off, wt.p + off, L.taps,
                                                                        L.cout, L.cin);
            off += cnt;
        }
        e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        return e;
    }

    hipError_t get(const float* src, float* host) {
        hipError_t e = hipMemcpyAsync(host, src, total_weights() * sizeof(float), hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        return e;
    }

    int64_t woff(int l) const {
        int64_t o = 0;
        for (int q = 0; q < l; ++q) o += layer_size(q);
        return o;
    }

    // Forward pass on r (n^3 doubles, device); lk: normalised log kappa or
    // null.  Result: FP32 channel 0 of `out`.  ctl (nullable) predicates all
    // kernels on the solver's stop flag.
    // train: also materialise the skip concatenations (the weight gradients
    // of w7 and w9 read them); inference reads them in place.
    void forward(const Ctl* ctl, const double* r, const bf16* lk, hipStream_t s, bool train = false) {
        const int S0 = S, S1 = S / 2, S2 = S / 4;
        k_sumsq<<<kSqBlocks, kCB, 0, s>>>(ctl, r, n * n * n, part.p);
        k_finish_sum<<<1, kRedBlock, 0, s>>>(ctl, part.p, kSqBlocks, n * n * n, 0, small.p);
        // the 16-channel input only for training (the weight gradient of
        // the first layer reads it); the first layer forms channels 0 and 1
        // from r itself
        if (train) k_pack_input<<<blocks((size_t)S0 * S0 * S0), kCB, 0, s>>>(ctl, r, small.p, lk, x0.p, n, S0);
        k_conv_in2<<<dim3(S0 / 16 + (S0 % 16 != 0), S0 / 4, (S0 / 4 + kIn2Slabs - 1) / kIn2Slabs), kCB, 0, s>>>(
            ctl, r, small.p, lk, n,
                                                                                 wb.p + woff(0), e1.p, S0);
        // the second layer also writes its 2x2x2 average pooling (p1)
        conv_launch<16, 0, 16, 3, 1, 0, 1>(ctl, nullptr, e1.p, wb.p + woff(1), e2.p, S0, s, nullptr, p1.p);
        conv<16, 32, 3, 1, 0>(ctl, p1.p, 2, e3.p, S1, s);
        conv_launch<32, 0, 32, 3, 1, 0, 1>(ctl, nullptr, e3.p, wb.p + woff(3), e4.p, S1, s, nullptr, p2.p);
        conv<32, 64, 3, 1, 0>(ctl, p2.p, 4, b1.p, S2, s);
        conv<64, 64, 3, 1, 0>(ctl, b1.p, 5, b2.p, S2, s);
        if (train) k_upcat<<<blocks((size_t)S1 * S1 * S1 * 96), kCB, 0, s>>>(ctl, b2.p, e4.p, c1.p, S1, 64, 32);
        conv_cat<96, 64, 32>(ctl, b2.p, e4.p, 6, d1.p, S1, s);
        conv<32, 32, 3, 1, 0>(ctl, d1.p, 7, d2.p, S1, s);
        if (train) k_upcat<<<blocks((size_t)S0 * S0 * S0 * 48), kCB, 0, s>>>(ctl, d2.p, e2.p, c2.p, S0, 32, 16);
        conv_cat<48, 32, 16>(ctl, d2.p, e2.p, 8, d3.p, S0, s);
        if (train) {
            conv<16, 16, 3, 1, 0>(ctl, d3.p, 9, d4.p, S0, s);
            conv<16, 16, 1, 0, 1>(ctl, d4.p, 10, out.p, S0, s);
        } else {
            // inference: the last 3x3x3 layer and the 1x1 output layer in one
            // pass (the 16-channel activation is not stored)
            conv_launch<16, 0, 16, 3, 1, 2>(ctl, nullptr, d3.p, wb.p + woff(9), out.p, S0, s, wb.p + woff(10));
        }
    }

    // Loss against e / rms(e) and all weight gradients into g (FP32).
    // MSE loss against e / rms(e): loss -> small[2], output gradient -> g0a.
    void loss_mse(const double* e, hipStream_t s) {
        const size_t V0 = (size_t)S * S * S;
        k_sumsq<<<kSqBlocks, kCB, 0, s>>>(nullptr, e, n * n * n, part.p);
        k_finish_sum<<<1, kRedBlock, 0, s>>>(nullptr, part.p, kSqBlocks, n * n * n, 0, small.p + 1);
        k_mse_grad<<<blocks(V0), kCB, 0, s>>>(out.p, e, small.p + 1, g0a.p, n, S, part.p);
        k_finish_sum<<<1, kRedBlock, 0, s>>>(nullptr, part.p, (int)blocks(V0), 0, 1, small.p + 2);
    }

    // The network output d on the n^3 nodes (FP64) -> dvec.
    void output_vector(hipStream_t s) {
        k_clear_flag<<<1, 64, 0, s>>>(nullptr, flag.p);
        k_unpack_output<double><<<blocks((size_t)n * n * n), kCB, 0, s>>>(nullptr, out.p, dvec.p, n, S, flag.p);
    }

    // Energy loss of dvec for (r, e) given q = A dvec (or their parts
    // A-orthogonal to a block): loss -> small[2], output gradient -> g0a.
    void loss_energy(const double* r, const double* q, const double* e, hipStream_t s) {
        k_dots3<<<kSumBlocks, kCB, 0, s>>>(dvec.p, q, r, e, n * n * n, part.p);
        k_energy_finish<<<1, kRedBlock, 0, s>>>(part.p, kSumBlocks, small.p + 4);
        k_energy_grad<<<blocks((size_t)S * S * S), kCB, 0, s>>>(small.p + 4, q, r, g0a.p, n, S);
        (void)hipMemcpyAsync(small.p + 2, small.p + 7, sizeof(double), hipMemcpyDeviceToDevice, s);
    }

    hipError_t read_loss(double* loss) {
        double h = 0.0;
        hipError_t err = hipGetLastError();
        if (err == hipSuccess) err = hipMemcpyAsync(&h, small.p + 2, sizeof(double), hipMemcpyDeviceToHost, stream);
        if (err == hipSuccess) err = hipStreamSynchronize(stream);
        if (loss) *loss = h;
        return err;
    }

    // Weight gradients into g (FP32) from the output gradient in g0a.
    void backward(hipStream_t s) {
        const int S0 = S, S1 = S / 2, S2 = S / 4;
        const size_t V0 = (size_t)S0 * S0 * S0, V1 = V0 / 8, V2 = V1 / 8;
        (void)hipMemsetAsync(g.p, 0, total_weights() * sizeof(float), s);
        // output layer (1x1)
        wgrad<16, 16, 1>(g0a.p, d4.p, 10, S0, s);
        dgrad<16, 16, 1>(g0a.p, 10, g0b.p, S0, s);                      // dd4
        mask(g0b.p, d4.p, g0a.p, V0 * 16, s);                            // dpre10
        wgrad<16, 16, 3>(g0a.p, d3.p, 9, S0, s);
        dgrad<16, 16, 3>(g0a.p, 9, g0b.p, S0, s);                       // dd3
        mask(g0b.p, d3.p, g0a.p, V0 * 16, s);                            // dpre9
        wgrad<48, 16, 3>(g0a.p, c2.p, 8, S0, s);
        dgrad<48, 16, 3>(g0a.p, 8, g0c.p, S0, s);                       // dc2 (48)
        k_upsample_bwd<<<blocks(V1 * 32), kCB, 0, s>>>(nullptr, g0c.p, g1b.p, S1, 32, 48);   // dd2
        mask(g1b.p, d2.p, g1c.p, V1 * 32, s);                            // dpre8
        wgrad<32, 32, 3>(g1c.p, d1.p, 7, S1, s);
        dgrad<32, 32, 3>(g1c.p, 7, g1b.p, S1, s);                       // dd1
        mask(g1b.p, d1.p, g1c.p, V1 * 32, s);                            // dpre7
        wgrad<96, 32, 3>(g1c.p, c1.p, 6, S1, s);
        dgrad<96, 32, 3>(g1c.p, 6, g1a.p, S1, s);                       // dc1 (96)
        k_upsample_bwd<<<blocks(V2 * 64), kCB, 0, s>>>(nullptr, g1a.p, g2a.p, S2, 64, 96);   // db2
        mask(g2a.p, b2.p, g2b.p, V2 * 64, s);                            // dpre6
        wgrad<64, 64, 3>(g2b.p, b1.p, 5, S2, s);
        dgrad<64, 64, 3>(g2b.p, 5, g2a.p, S2, s);                       // db1
        mask(g2a.p, b1.p, g2b.p, V2 * 64, s);                            // dpre5
        wgrad<32, 64, 3>(g2b.p, p2.p, 4, S2, s);
        dgrad<32, 64, 3>(g2b.p, 4, g2c.p, S2, s);                       // dp2
        k_skip_pool_bwd<<<blocks(V1 * 32), kCB, 0, s>>>(nullptr, g1a.p, g2c.p, g1b.p, S1, 64, 32);  // de4
        mask(g1b.p, e4.p, g1c.p, V1 * 32, s);                            // dpre4
        wgrad<32, 32, 3>(g1c.p, e3.p, 3, S1, s);
        dgrad<32, 32, 3>(g1c.p, 3, g1b.p, S1, s);                       // de3
        mask(g1b.p, e3.p, g1c.p, V1 * 32, s);                            // dpre3
        wgrad<16, 32, 3>(g1c.p, p1.p, 2, S1, s);
        dgrad<16, 32, 3>(g1c.p, 2, g1b.p, S1, s);                       // dp1 (16 ch)
        k_skip_pool_bwd<<<blocks(V0 * 16), kCB, 0, s>>>(nullptr, g0c.p, g1b.p, g0b.p, S0, 32, 16);  // de2
        mask(g0b.p, e2.p, g0a.p, V0 * 16, s);                            // dpre2
        wgrad<16, 16, 3>(g0a.p, e1.p, 1, S0, s);
        dgrad<16, 16, 3>(g0a.p, 1, g0b.p, S0, s);                       // de1
        mask(g0b.p, e1.p, g0a.p, V0 * 16, s);                            // dpre1
        wgrad<16, 16, 3>(g0a.p, x0.p, 0, S0, s);
    }

    // Stand-alone inference: d (n^3 doubles) = N(r); *finite = no NaN/Inf.
    hipError_t infer(const double* r, const bf16* lk, double* d, bool* finite) {
        forward(nullptr, r, lk, stream);
        k_clear_flag<<<1, 64, 0, stream>>>(nullptr, flag.p);
        k_unpack_output<double><<<blocks((size_t)n * n * n), kCB, 0, stream>>>(nullptr, out.p, d, n, S, flag.p);
        int f = 0;
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(&f, flag.p, sizeof(int), hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (finite) *finite = f == 0;
        return e;
    }

    // Loss and weight gradients for one pair (r, e); with lr > 0 also one
    // Adam step.  Synchronises to return the loss.
    hipError_t step_pair(const double* r, const bf16* lk, const double* e, float lr, double* loss) {
        forward(nullptr, r, lk, stream, true);
        loss_mse(e, stream);
        backward(stream);
        if (lr > 0.f) adam(lr, stream);
        return read_loss(loss);
    }

    void adam(float lr, hipStream_t s) {
        ++step;
        const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
        const float c1 = 1.f - std::pow(b1, (float)step), c2 = 1.f - std::pow(b2, (float)step);
        int64_t off = 0;
        for (int l = 0; l < 11; ++l) {
            const LayerSpec L = kLayers[l];
            const int cnt = (int)layer_size(l);
            k_adam<<<(cnt + kCB - 1) / kCB, kCB, 0, s>>>(w.p + off, m.p + off, v.p + off, g.p + off, wb.p + off,
                                                          wt.p + off, L.taps, L.cout, L.cin, lr, b1, b2, eps, c1,
                                                          c2);
            off += cnt;
        }
    }

    Buf<bf16> x0, e1, e2, p1, e3, e4, p2, b1, b2, c1, d1, d2, c2, d3, d4;
    Buf<float> out;
    Buf<bf16> g0a, g0b, g0c, g1a, g1b, g1c, g2a, g2b, g2c;
    Buf<double> small, part, dvec, qvec, rvec, q2vec;
    Buf<int> flag;
    Buf<float> w, m, v, g;
    Buf<bf16> wb, wt;
    int step = 0;

    // One layer on caller tensors (S^3 grid, channels-last bfloat16) with
    // the current weights.  op 0: out = relu(conv(A)) (layer 11: FP32 output
    // channel 0, no ReLU); op 1: out = data gradient of output gradient A; op 2: out (FP32,
    // the layer's weight count) = weight gradient of output gradient A and
    // layer input B.
    hipError_t layer_op(int l, int op, int Sg, const bf16* A, const bf16* B, void* out) {
        switch (l) {
            case 0: layer_t<16, 16, 3, 0>(l, op, Sg, A, B, out); break;
            case 1: layer_t<16, 16, 3, 0>(l, op, Sg, A, B, out); break;
            case 2: layer_t<16, 32, 3, 0>(l, op, Sg, A, B, out); break;
            case 3: layer_t<32, 32, 3, 0>(l, op, Sg, A, B, out); break;
            case 4: layer_t<32, 64, 3, 0>(l, op, Sg, A, B, out); break;
            case 5: layer_t<64, 64, 3, 0>(l, op, Sg, A, B, out); break;
            case 6: layer_t<96, 32, 3, 0>(l, op, Sg, A, B, out); break;
            case 7: layer_t<32, 32, 3, 0>(l, op, Sg, A, B, out); break;
            case 8: layer_t<48, 16, 3, 0>(l, op, Sg, A, B, out); break;
            case 9: layer_t<16, 16, 3, 0>(l, op, Sg, A, B, out); break;
            default: layer_t<16, 16, 1, 1>(l, op, Sg, A, B, out); break;
        }
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        return e;
    }

   private:
    static unsigned blocks(size_t count) { return (unsigned)((count + kCB - 1) / kCB); }

    template <int CIN, int COUT, int KS, int LAST>
    void layer_t(int l, int op, int Sg, const bf16* A, const bf16* B, void* out) {
        if (op == 0) {
            conv_p<CIN, COUT, KS, LAST ? 0 : 1, LAST>(nullptr, A, wb.p + woff(l), out, Sg, stream);
        } else if (op == 1) {
            dgrad_p<CIN, COUT, KS>(A, wt.p + woff(l), static_cast<bf16*>(out), Sg, stream);
        } else {
            (void)hipMemsetAsync(out, 0, layer_size(l) * sizeof(float), stream);
            wgrad_p<CIN, COUT, KS>(A, B, static_cast<float*>(out), Sg, stream);
        }
    }

    static dim3 conv_grid(int Sg, int split, int ty) {
        return dim3((Sg + 15) / 16, (Sg + ty - 1) / ty, ((Sg + 3) / 4) * split);
    }

    // Small grids (fewer than kConvFill tiles) split the output channels
    // over blocks so that the whole chip works.
    static constexpr int kConvFill = 1024;
    // POOL: also the 2x2x2 average pooling of the output into Yp (grid Sg/2)
    template <int CIN, int C1, int COUT, int KS, int RELU, int F32, int POOL = 0>
    static void conv_launch(const Ctl* ctl, const bf16* Xc, const bf16* X, const bf16* Wl, void* Y, int Sg,
                            hipStream_t s, const bf16* W2 = nullptr, bf16* Yp = nullptr) {
        const int tiles = ((Sg + 15) / 16) * ((Sg + conv_ty<CIN>() - 1) / conv_ty<CIN>()) * ((Sg + 3) / 4);
        if constexpr (!F32 && COUT % 64 == 0) {
            if (tiles < kConvFill) {
                k_conv_lds<CIN, C1, COUT, KS, RELU, F32, 4, POOL><<<conv_grid(Sg, 4, conv_ty<CIN>()), kCB, 0, s>>>(
                    ctl, Xc, X, Wl, Y, Sg, W2, Yp);
                return;
            }
        }
        if constexpr (!F32 && COUT % 32 == 0) {
            if (tiles < kConvFill) {
                k_conv_lds<CIN, C1, COUT, KS, RELU, F32, 2, POOL><<<conv_grid(Sg, 2, conv_ty<CIN>()), kCB, 0, s>>>(
                    ctl, Xc, X, Wl, Y, Sg, W2, Yp);
                return;
            }
        }
        k_conv_lds<CIN, C1, COUT, KS, RELU, F32, 1, POOL><<<conv_grid(Sg, 1, conv_ty<CIN>()), kCB, 0, s>>>(
            ctl, Xc, X, Wl, Y, Sg, W2, Yp);
    }

    template <int CIN, int COUT, int KS, int RELU, int F32>
    static void conv_p(const Ctl* ctl, const bf16* X, const bf16* Wl, void* Y, int Sg, hipStream_t s) {
        conv_launch<CIN, 0, COUT, KS, RELU, F32>(ctl, nullptr, X, Wl, Y, Sg, s);
    }
    // data gradient of a layer (CIN, COUT): the forward kernel on the
    // flipped, transposed weights, input dY (COUT channels) -> dX (CIN)
    template <int CIN, int COUT, int KS>
    static void dgrad_p(const bf16* dY, const bf16* Wt, bf16* dX, int Sg, hipStream_t s) {
        conv_launch<COUT, 0, CIN, KS, 0, 0>(nullptr, nullptr, dY, Wt, dX, Sg, s);
    }
    // conv + ReLU of [upsample2(Xc) (C1 channels) | X] without forming the concatenation
    template <int CIN, int C1, int COUT>
    void conv_cat(const Ctl* ctl, const bf16* Xc, const bf16* X, int layer, bf16* Y, int Sg, hipStream_t s) {
        conv_launch<CIN, C1, COUT, 3, 1, 0>(ctl, Xc, X, wb.p + woff(layer), Y, Sg, s);
    }
    template <int CIN, int COUT, int KS>
    static void wgrad_p(const bf16* dY, const bf16* X, float* dW, int Sg, hipStream_t s) {
        const int tiles = Sg * Sg * ((Sg + 15) / 16);
        const int per = 256;
        dim3 grid((tiles + per - 1) / per, KS == 3 ? 27 : 1);
        k_conv_wgrad<CIN, COUT, KS><<<grid, kCB, 0, s>>>(nullptr, dY, X, dW, Sg, per);
    }

    template <int CIN, int COUT, int KS, int RELU, int F32>
    void conv(const Ctl* ctl, const bf16* X, int layer, void* Y, int Sg, hipStream_t s) {
        conv_p<CIN, COUT, KS, RELU, F32>(ctl, X, wb.p + woff(layer), Y, Sg, s);
    }
    template <int CIN, int COUT, int KS>
    void dgrad(const bf16* dY, int layer, bf16* dX, int Sg, hipStream_t s) {
        dgrad_p<CIN, COUT, KS>(dY, wt.p + woff(layer), dX, Sg, s);
    }
    template <int CIN, int COUT, int KS>
    void wgrad(const bf16* dY, const bf16* X, int layer, int Sg, hipStream_t s) {
        wgrad_p<CIN, COUT, KS>(dY, X, g.p + woff(layer), Sg, s);
    }
    void mask(const bf16* dpost, const bf16* post, bf16* dpre, size_t count, hipStream_t s) {
        k_relu_mask<<<blocks(count), kCB, 0, s>>>(nullptr, dpost, post, dpre, count);
    }
};

// net.forward(ctl, r, lk, s), compiled once (with the rest of the network's
// kernels) rather than in every solver translation unit.
void net_forward(Net& net, const Ctl* ctl, const double* r, const bf16* lk, hipStream_t s);

}  // namespace cnn
}  // namespace amg
