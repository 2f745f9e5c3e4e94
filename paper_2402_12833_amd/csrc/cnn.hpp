// Learned search direction: a 3-level U-Net (16/32/64 channels, 3x3x3
// convolutions, no bias, ReLU, 2x average pooling, nearest upsampling with
// skip concatenation, 1x1 output) whose output is appended to the MPCG block
// as one more direction, so the energy minimisation decides its coefficient.
//
// Tensors are channels-last bfloat16 on an S^3 grid (S a multiple of 4 that
// holds the n^3 problem grid in its low corner): t[((z*S + y)*S + x)*C + c].
// Convolutions are implicit GEMMs on the matrix cores: M = voxels (16 along
// x per M tile), N = output channels, K = taps x input channels, with
// v_mfma_f32_16x16x32_bf16 (forward and data gradient, input tiles staged in
// LDS) and v_mfma_f32_16x16x16_bf16 (weight gradient), FP32 accumulation.
// Weights: bfloat16 copies [tap][Cout][Cin] of FP32 masters (Adam).  The
// backward data gradient is the same forward kernel on the tap-flipped,
// channel-transposed weights; weight gradients are GEMMs over voxels
// accumulated with FP32 atomics.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace amg {
namespace cnn {

using bf16 = unsigned short;
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bfloat16, round to nearest even
__device__ __forceinline__ bf16 f2bf(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (bf16)(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16 h) { return __uint_as_float((unsigned)h << 16); }

__host__ __device__ constexpr int tap_dz(int t) { return t / 9 - 1; }
__host__ __device__ constexpr int tap_dy(int t) { return (t / 3) % 3 - 1; }
__host__ __device__ constexpr int tap_dx(int t) { return t % 3 - 1; }

constexpr int kCB = 256;   // threads per block of the CNN kernels (4 wavefronts)

// ------------------------------------------------------------- convolution
// Y[v, co] = sum_t sum_ci X[v + o_t, ci] W[t, co, ci] (zero outside the grid).

typedef short bf16x8 __attribute__((ext_vector_type(8)));

// LDS-tiled convolution.  A block computes a 16 (x) x TY (y) x 4 (z) tile of
// output voxels, one z plane per wavefront and TY 16-voxel rows per
// wavefront, for COUT / CSPLIT output channels (blockIdx.z also selects the
// channel slice).  The input tile with its one-voxel halo is staged in LDS
// once per chunk of CC input channels, row by row: each thread keeps one
// (x, 8-channel piece) column of the tile rows and walks the rows, so the
// index arithmetic per 16-byte piece is a few adds.  K (taps x channels) is
// walked with v_mfma_f32_16x16x32_bf16 with the weights as the M operand
// (16 output channels) and the input as the N operand (16 voxels along x): a
// step fixes, per lane group kq, one (dz, dx) offset and 8 channels (CC = 32:
// one offset, channels 8 kq..; CC = 16: two offsets, lane groups 0-1 and
// 2-3), reads the fragments of the TY + 2 input rows once and uses row
// y0 + i + dy for output row i and tap dy, so each fragment serves three
// taps.  Both operands use the same K assignment, so the sum does not depend
// on the hardware's K order.  Each lane then holds 4 consecutive output
// channels of one voxel: the epilogue converts them pairwise to bfloat16
// (round to nearest even) and writes 8 bytes per lane.  Input channels
// c < C1 come from Xc, a grid of S/2 read at (z/2, y/2, x/2) (nearest
// upsampling), the rest from X (CIN - C1 channels): the skip concatenation
// is read in place.  OUT_F32 = 1: FP32 output of channel 0 only, one value per
// voxel (the network output layer).  OUT_F32 = 2 (16 output channels in one
// block): the network's last two layers at once, the ReLU output rounded to
// bfloat16 as if stored, then the 1x1 output layer W2 (channel 0 of its
// [16][16] weights) summed over the 16 channels in FP32 (per lane its 4
// channels, then the 4 lane groups), one FP32 value per voxel.
// Output rows (y) per wavefront.  4: with 8 (fewer fragment reads per MFMA)
// the LDS tile of a 16-channel chunk grows to 52 KB, three blocks per CU
// instead of five, and the layers ran slower (52 -> 57 us at 128^3).
template <int CIN>
__host__ __device__ constexpr int conv_ty() { return 4; }

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef short i16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ unsigned pack_bf16x2(float lo, float hi) {
    const bf16x2_t v = __builtin_convertvector(f32x2_t{lo, hi}, bf16x2_t);
    return __builtin_bit_cast(unsigned, v);
}

template <int CIN, int C1, int COUT, int KS, int RELU, int OUT_F32, int CSPLIT, int POOL = 0>
__global__ void __launch_bounds__(kCB) k_conv_lds(const Ctl* __restrict__ ctl, const bf16* __restrict__ Xc,
                                                  const bf16* __restrict__ X, const bf16* __restrict__ W,
                                                  void* __restrict__ Yv, int S, const bf16* __restrict__ W2,
                                                  bf16* __restrict__ Yp) {
    if (ctl && ctl->state != 0) return;
    static_assert(!POOL || (OUT_F32 == 0 && KS == 3 && conv_ty<CIN>() == 4), "pooling: bfloat16 3x3x3 layers");
    static_assert(CIN % 16 == 0 && COUT % (16 * CSPLIT) == 0 && C1 % 16 == 0 && C1 < CIN, "channel layout");
    static_assert(OUT_F32 != 2 || COUT / CSPLIT == 16, "the fused output layer needs all 16 channels in one block");
    constexpr int C2 = CIN - C1;
    constexpr int CC = (CIN % 32 == 0) ? 32 : 16;      // channels per LDS stage
    constexpr int NCH = CIN / CC;
    constexpr int H = KS == 3 ? 1 : 0;
    constexpr int TY = conv_ty<CIN>();
    constexpr int LX = 16 + 2 * H, LY = TY + 2 * H, LZ = 4 + 2 * H;
    constexpr int NV = LX * LY * LZ;
    constexpr int VS = CC + 8;                         // padded voxel stride (elements)
    constexpr int NT = COUT / 16 / CSPLIT;
    constexpr int NCOMBO = KS == 3 ? 9 : 1;            // (dz, dx) offsets
    constexpr int NSTEP = CC == 32 ? NCOMBO : (NCOMBO + 1) / 2;
    constexpr int NDY = KS == 3 ? 3 : 1;
    constexpr int PIECES = CC / 8;                     // 16-byte pieces per voxel and stage
    constexpr int PR = LX * PIECES;                    // pieces per tile row
    constexpr int NR = LY * LZ;                        // tile rows
    constexpr int RPP = kCB / PR;                      // tile rows per staging pass
    __shared__ __attribute__((aligned(16))) bf16 tile[NV * VS];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int m = lane & 15, kq = lane >> 4;
    const int ztiles = (S + 3) >> 2;
    const int zt = blockIdx.z % ztiles, cs = blockIdx.z / ztiles;
    const int x0 = blockIdx.x * 16, y0 = blockIdx.y * TY, z0 = zt * 4;
    const int co0 = cs * NT * 16;
    const int Sc = S >> 1;
    // this thread's staging column: x = slx of the tile, 8 channels from sq * 8
    const int srow = threadIdx.x / PR, scol = threadIdx.x - srow * PR;
    const int slx = scol / PIECES, sq = scol % PIECES;
    const int gx = x0 - H + slx;
    const bool xin = srow < RPP && gx >= 0 && gx < S;
    // per-lane parts of the fragment addresses: lane group kq reads channels
    // cl.. (lane half hb: the second offset of a CC = 16 step); tl: this
    // lane's input for output row 0 at offset 0
    const int cl = CC == 32 ? 8 * kq : 8 * (kq & 1);
    const bool hb = CC == 16 && (kq >> 1) != 0;
    const bf16* const tl = tile + (((w + H) * LY) * LX + (m + H)) * VS + cl;
    const unsigned wbase = (unsigned)((co0 + m) * CIN + cl);
    const char* const Wb = reinterpret_cast<const char*>(W);
    f32x4 acc[TY][NT];
#pragma unroll
    for (int i = 0; i < TY; ++i)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[i][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    // the 16-byte pieces of this thread's column of chunk ch: rows srow,
    // srow + RPP, .. (at most NPASS).  With 32-channel chunks (their LDS
    // tile already limits a CU to three blocks, so the registers are there)
    // the next chunk's pieces are loaded during the current chunk's MFMAs.
    constexpr int NPASS = (NR + RPP - 1) / RPP;
    int4 stg[NPASS];
    auto stage_load = [&](int ch) {
        const int c = ch * CC + sq * 8;
#pragma unroll
        for (int t = 0; t < NPASS; ++t) {
            const int r = srow + t * RPP;
            const int ly = r % LY, lz = r / LY;
            const int gy = y0 - H + ly, gz = z0 - H + lz;
            int4 val = int4{0, 0, 0, 0};
            if (r < NR && xin && gy >= 0 && gy < S && gz >= 0 && gz < S) {
                // 32-bit byte offsets from the (uniform) array bases
                if (c < C1)
                    val = *reinterpret_cast<const int4*>(
                        reinterpret_cast<const char*>(Xc) +
                        2u * (unsigned)((((gz >> 1) * Sc + (gy >> 1)) * Sc + (gx >> 1)) * C1 + c));
                else
                    val = *reinterpret_cast<const int4*>(reinterpret_cast<const char*>(X) +
                                                         2u * (unsigned)(((gz * S + gy) * S + gx) * C2 + (c - C1)));
            }
            stg[t] = val;
        }
    };
    constexpr bool kPre = CC == 32;
    stage_load(0);
    for (int ch = 0; ch < NCH; ++ch) {
        if (ch > 0) __syncthreads();   // the previous chunk's MFMAs are done with the tile
        if (!kPre && ch > 0) stage_load(ch);
        if (srow < RPP) {
#pragma unroll
            for (int t = 0; t < NPASS; ++t) {
                const int r = srow + t * RPP;
                if (r < NR) *reinterpret_cast<int4*>(tile + (r * LX + slx) * VS + sq * 8) = stg[t];
            }
        }
        __syncthreads();
        if (kPre && ch + 1 < NCH) stage_load(ch + 1);
        // step st's (dz, dx) offset: one for all lanes (CC = 32), or one per
        // lane half (CC = 16; combo 9 of the last step is past the taps: its
        // weights are zero, its input any valid row); the weights of step
        // st + 1 are loaded during step st
        auto combo_of = [&](int st, int& dz, int& dx, bool& none) {
            const int cA = CC == 32 ? st : 2 * st, cB = CC == 32 ? st : 2 * st + 1;
            const int c = hb ? cB : cA;
            none = c >= NCOMBO;
            const int cv = none ? 0 : c;
            dz = KS == 3 ? cv / 3 - 1 : 0;
            dx = KS == 3 ? cv % 3 - 1 : 0;
        };
        auto load_w = [&](int st, bf16x8 (&b)[NDY][NT]) {
            int dz, dx;
            bool none;
            combo_of(st, dz, dx, none);
#pragma unroll
            for (int dyi = 0; dyi < NDY; ++dyi) {
                const int dy = KS == 3 ? dyi - 1 : 0;
                const int tap = KS == 3 ? (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1) : 0;
                const unsigned woff = wbase + (unsigned)(tap * COUT * CIN + ch * CC);
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    b[dyi][nt] = *reinterpret_cast<const bf16x8*>(Wb + 2u * (woff + (unsigned)(nt * 16 * CIN)));
                    if (none) b[dyi][nt] = bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
                }
            }
        };
        bf16x8 bw[2][NDY][NT];
        load_w(0, bw[0]);
#pragma unroll
        for (int st = 0; st < NSTEP; ++st) {
            int dz, dx;
            bool none;
            combo_of(st, dz, dx, none);
            const int voff = dz * LY * LX + dx;
            bf16x8 a[TY + 2 * H];
#pragma unroll
            for (int r = 0; r < TY + 2 * H; ++r)
                a[r] = *reinterpret_cast<const bf16x8*>(tl + (voff + r * LX) * VS);
            if (st + 1 < NSTEP) load_w(st + 1, bw[(st + 1) & 1]);
            // keep those loads here: the scheduler would otherwise sink them
            // next to their first use and wait for them there
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int dyi = 0; dyi < NDY; ++dyi) {
                const int dy = KS == 3 ? dyi - 1 : 0;
#pragma unroll
                for (int i = 0; i < TY; ++i)
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt)
                        acc[i][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bw[st & 1][dyi][nt], a[i + dy + H],
                                                                             acc[i][nt], 0, 0, 0);
            }
        }
    }
    // lane (m, kq): voxel x0 + m, channels co0 + nt * 16 + 4 kq .. + 3
    const int z = z0 + w, x = x0 + m;
    const bool vin = z < S && x < S;
    char* const Yb = static_cast<char*>(Yv);
    if constexpr (OUT_F32 != 0) {
        if (!vin) return;
#pragma unroll
        for (int i = 0; i < TY; ++i) {
            const int y = y0 + i;
            if (y >= S) break;
            const unsigned vox = (unsigned)((z * S + y) * S + x);
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int co = co0 + nt * 16 + 4 * kq;
                if (OUT_F32 == 2) {
                    // the activation as stored: bfloat16 pairs (round to
                    // nearest even), ReLU as a 16-bit integer max, then back
                    // to FP32 for the dot product with the output weights
                    i16x2 p0 = __builtin_bit_cast(i16x2, pack_bf16x2(acc[i][nt][0], acc[i][nt][1]));
                    i16x2 p1 = __builtin_bit_cast(i16x2, pack_bf16x2(acc[i][nt][2], acc[i][nt][3]));
                    if (RELU) {
                        p0 = __builtin_elementwise_max(p0, i16x2{0, 0});
                        p1 = __builtin_elementwise_max(p1, i16x2{0, 0});
                    }
                    const unsigned u0 = __builtin_bit_cast(unsigned, p0), u1 = __builtin_bit_cast(unsigned, p1);
                    const float v[4] = {__uint_as_float(u0 << 16), __uint_as_float(u0 & 0xffff0000u),
                                        __uint_as_float(u1 << 16), __uint_as_float(u1 & 0xffff0000u)};
                    float part = 0.f;
#pragma unroll
                    for (int j = 0; j < 4; ++j) part += v[j] * bf2f(W2[co + j]);
                    part += __shfl_xor(part, 16);
                    part += __shfl_xor(part, 32);
                    if (kq == 0) *reinterpret_cast<float*>(Yb + 4u * vox) = part;
                } else {
                    float v = acc[i][nt][0];
                    if (RELU) v = v > 0.f ? v : 0.f;
                    if (co == 0) *reinterpret_cast<float*>(Yb + 4u * vox) = v;
                }
            }
        }
    } else {
        // ReLU on the bfloat16 pairs as signed 16-bit integers: a negative
        // value (sign bit set) is below 0 and becomes +0
        uint2 pk[TY][NT];
#pragma unroll
        for (int i = 0; i < TY; ++i)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                i16x2 p0 = __builtin_bit_cast(i16x2, pack_bf16x2(acc[i][nt][0], acc[i][nt][1]));
                i16x2 p1 = __builtin_bit_cast(i16x2, pack_bf16x2(acc[i][nt][2], acc[i][nt][3]));
                if (RELU) {
                    p0 = __builtin_elementwise_max(p0, i16x2{0, 0});
                    p1 = __builtin_elementwise_max(p1, i16x2{0, 0});
                }
                pk[i][nt].x = __builtin_bit_cast(unsigned, p0);
                pk[i][nt].y = __builtin_bit_cast(unsigned, p1);
            }
        if (vin) {
#pragma unroll
            for (int i = 0; i < TY; ++i) {
                const int y = y0 + i;
                if (y >= S) break;
                const unsigned vox = (unsigned)((z * S + y) * S + x);
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    *reinterpret_cast<uint2*>(Yb + 2u * (vox * COUT + (unsigned)(co0 + nt * 16 + 4 * kq))) = pk[i][nt];
            }
        }
        if constexpr (POOL) {
            // 2x2x2 average pooling of the stored (bfloat16) outputs into Yp
            // (grid S/2): the block's 16 x 4 x 4 voxels are 8 x 2 x 2 coarse
            // voxels; the outputs go through LDS (the tile is free once every
            // wavefront is past its MFMAs), then each thread sums the 8
            // children of one coarse voxel and 2 channels in FP32 in (z, y,
            // x) order, scales by 1/8 and rounds to bfloat16.
            constexpr int CB = NT * 16;
            static_assert(4 * TY * 16 * CB <= NV * VS, "pool staging fits in the tile");
            __syncthreads();
            unsigned* const pw = reinterpret_cast<unsigned*>(tile);
#pragma unroll
            for (int i = 0; i < TY; ++i)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    *reinterpret_cast<uint2*>(pw + ((w * TY + i) * 16 + m) * (CB / 2) + nt * 8 + 2 * kq) = pk[i][nt];
            __syncthreads();
            const int Sc = S >> 1;
            for (int q = threadIdx.x; q < 32 * (CB / 2); q += kCB) {
                const int c2 = q % (CB / 2), cv = q / (CB / 2);
                const int xc = cv & 7, yc = (cv >> 3) & 1, zc = cv >> 4;
                const int gxc = (x0 >> 1) + xc, gyc = (y0 >> 1) + yc, gzc = (z0 >> 1) + zc;
                if (gxc >= Sc || gyc >= Sc || gzc >= Sc) continue;
                float s0 = 0.f, s1 = 0.f;
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
#pragma unroll
                        for (int d = 0; d < 2; ++d) {
                            const unsigned u = pw[(((2 * zc + a) * TY + 2 * yc + b) * 16 + 2 * xc + d) * (CB / 2) + c2];
                            s0 += bf2f((bf16)(u & 0xffffu));
                            s1 += bf2f((bf16)(u >> 16));
                        }
                const unsigned o = (unsigned)f2bf(s0 * 0.125f) | ((unsigned)f2bf(s1 * 0.125f) << 16);
                *reinterpret_cast<unsigned*>(Yp + ((size_t)(gzc * Sc + gyc) * Sc + gxc) * COUT + co0 + 2 * c2) = o;
            }
        }
    }
}

constexpr int kIn2Slabs = 4;   // 4-plane z slabs per block of k_conv_in2

// The network's first layer (3x3x3, 16 outputs, ReLU) on its input, whose
// channels 2..15 are zero: K = 27 taps x 2 channels (54, padded to 64 = two
// v_mfma_f32_16x16x32_bf16 steps instead of 14 over the zero channels).  The
// input is formed while the tile is staged, as k_pack_input forms it:
// channel 0 = bfloat16(r * scale) from the n^3 FP64 vector r, channel 1 =
// lk (or 0), both 0 outside n^3; one 32-bit word per voxel in LDS.  W: the
// layer's weights [tap][16][16] of which channels 0 and 1 are read.  K slot k of a step:
// tap 16 st + k / 2, channel k % 2; lane group kq holds slots 8 kq .. 8 kq + 7
// (taps 16 st + 4 kq + j, j = 0..3) for both operands, so the sum does not
// depend on the hardware's K order.  Tile, wavefront rows and epilogue as in
// k_conv_lds.
static __global__ void __launch_bounds__(kCB) k_conv_in2(const Ctl* __restrict__ ctl, const double* __restrict__ r,
                                                  const double* __restrict__ scale, const bf16* __restrict__ lk,
                                                  int n, const bf16* __restrict__ W, bf16* __restrict__ Y, int S) {
    if (ctl && ctl->state != 0) return;
    constexpr int LX = 18, LY = 6, LZ = 6, NV = LX * LY * LZ, NIT = (NV + kCB - 1) / kCB;
    __shared__ unsigned tile[NV];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int m = lane & 15, kq = lane >> 4;
    const int x0 = blockIdx.x * 16, y0 = blockIdx.y * 4;
    const float sc = (float)(*scale);
    // this thread's tile voxels (v = threadIdx.x + q kCB): fixed (x, y),
    // z offset from the slab's first plane
    int toffs[NIT], tz[NIT];
    bool txy[NIT];
#pragma unroll
    for (int q = 0; q < NIT; ++q) {
        const int v = threadIdx.x + q * kCB;
        const int lx = v % LX, ly = (v / LX) % LY, lz = v / (LX * LY);
        const int gx = x0 - 1 + lx, gy = y0 - 1 + ly;
        txy[q] = v < NV && gx >= 0 && gx < n && gy >= 0 && gy < n;
        toffs[q] = gx + n * gy;
        tz[q] = lz - 1;
    }
    // the slab's loads: all issued before any use
    double rv[NIT];
    bf16 kv[NIT];
    auto load_slab = [&](int z0) {
#pragma unroll
        for (int q = 0; q < NIT; ++q) {
            const int gz = z0 + tz[q];
            const bool in = txy[q] && gz >= 0 && gz < n;
            const int idx = in ? toffs[q] + n * n * gz : 0;
            rv[q] = in ? r[idx] : 0.0;
            kv[q] = (in && lk) ? lk[idx] : (bf16)0;
        }
    };
    // this lane's 4 taps per step: weights (channels 0, 1) and tile offsets
    typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
    u32x4 bw[2];
    int toff[2][4];
#pragma unroll
    for (int st = 0; st < 2; ++st)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int t = 16 * st + 4 * kq + j;
            const int tv = t < 27 ? t : 0;
            toff[st][j] = (tap_dz(tv) + 1) * LY * LX + (tap_dy(tv) + 1) * LX + (tap_dx(tv) + 1);
            bw[st][j] = t < 27 ? *reinterpret_cast<const unsigned*>(W + (size_t)(t * 16 + m) * 16) : 0u;
        }
    const unsigned* tl = tile + (w * LY) * LX + m;   // output row 0 of this wavefront at tap (-1, -1, -1)
    char* const Yb = reinterpret_cast<char*>(Y);
    const int x = x0 + m;
    // blockIdx.z: a group of kIn2Slabs consecutive 4-plane slabs; the next
    // slab's input is loaded during this slab's MFMAs and stores
    const int zs0 = blockIdx.z * kIn2Slabs;
    load_slab(zs0 * 4);
    for (int k = 0; k < kIn2Slabs; ++k) {
        const int z0 = (zs0 + k) * 4;
        if (z0 >= S) break;
        if (k > 0) __syncthreads();   // the previous slab's MFMAs are done with the tile
#pragma unroll
        for (int q = 0; q < NIT; ++q) {
            const int v = threadIdx.x + q * kCB;
            if (v < NV) tile[v] = (unsigned)f2bf((float)rv[q] * sc) | ((unsigned)kv[q] << 16);
        }
        __syncthreads();
        if (k + 1 < kIn2Slabs && z0 + 4 < S) load_slab(z0 + 4);
        f32x4 acc[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int st = 0; st < 2; ++st)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                u32x4 a;
#pragma unroll
                for (int j = 0; j < 4; ++j) a[j] = tl[toff[st][j] + i * LX];
                acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, bw[st]),
                                                                __builtin_bit_cast(bf16x8, a), acc[i], 0, 0, 0);
            }
        const int z = z0 + w;
        if (z < S && x < S) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int y = y0 + i;
                if (y >= S) break;
                const unsigned vox = (unsigned)((z * S + y) * S + x);
                i16x2 p0 = __builtin_bit_cast(i16x2, pack_bf16x2(acc[i][0], acc[i][1]));
                i16x2 p1 = __builtin_bit_cast(i16x2, pack_bf16x2(acc[i][2], acc[i][3]));
                p0 = __builtin_elementwise_max(p0, i16x2{0, 0});
                p1 = __builtin_elementwise_max(p1, i16x2{0, 0});
                uint2 pk;
                pk.x = __builtin_bit_cast(unsigned, p0);
                pk.y = __builtin_bit_cast(unsigned, p1);
                *reinterpret_cast<uint2*>(Yb + 2u * (vox * 16u + 4u * kq)) = pk;
            }
        }
    }
}

// dW[t, co, ci] += sum over voxels of dY[v, co] X[v + o_t, ci]; block = one
// tap and a range of 16-voxel x-tiles; lane l supplies A[m = co][k = voxel
// 4(l/16)+j] and B[k][n = ci]; each wavefront adds its sums with FP32 atomics.
template <int CIN, int COUT, int KS>
__global__ void __launch_bounds__(kCB) k_conv_wgrad(const Ctl* __restrict__ ctl, const bf16* __restrict__ dY,
                                                    const bf16* __restrict__ X, float* __restrict__ dW, int S,
                                                    int tiles_per_block) {
    if (ctl && ctl->state != 0) return;
    constexpr int MT = COUT / 16, NTI = CIN / 16, TAPS = KS == 3 ? 27 : 1;
    const int t = blockIdx.y;
    if (t >= TAPS) return;
    const int dz = KS == 3 ? tap_dz(t) : 0, dy = KS == 3 ? tap_dy(t) : 0, dx = KS == 3 ? tap_dx(t) : 0;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int m = lane & 15, kq = lane >> 4;
    const int xtiles = (S + 15) >> 4;
    const int ntiles = S * S * xtiles;
    f32x4 acc[MT][NTI];
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
        for (int b = 0; b < NTI; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int t0 = blockIdx.x * tiles_per_block;
    const int t1 = min(ntiles, t0 + tiles_per_block);
    for (int tile = t0 + wv; tile < t1; tile += kCB / 64) {
        const int row = tile / xtiles, xt = tile - row * xtiles;
        const int y = row % S, z = row / S, x0 = xt * 16;
        const int zz = z + dz, yy = y + dy;
        const bool rowok = zz >= 0 && zz < S && yy >= 0 && yy < S;
        bf16x4 af[MT], bfr[NTI];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int x = x0 + kq * 4 + j;          // the voxel of k = 4 kq + j
            const bool vin = x < S;
            const size_t vo = ((size_t)(z * S + y) * S + (vin ? x : 0)) * COUT;
#pragma unroll
            for (int a = 0; a < MT; ++a) af[a][j] = vin ? (short)dY[vo + a * 16 + m] : (short)0;
            const int xs = x + dx;
            const bool xin = vin && rowok && xs >= 0 && xs < S;
            const size_t xo = xin ? ((size_t)(zz * S + yy) * S + xs) * CIN : 0;
#pragma unroll
            for (int b = 0; b < NTI; ++b) bfr[b][j] = xin ? (short)X[xo + b * 16 + m] : (short)0;
        }
#pragma unroll
        for (int a = 0; a < MT; ++a)
#pragma unroll
            for (int b = 0; b < NTI; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[a], bfr[b], acc[a][b], 0, 0, 0);
    }
    // D[m = co (4 kq + j)][n = ci (lane % 16)]
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
        for (int b = 0; b < NTI; ++b)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int co = a * 16 + kq * 4 + j, ci = b * 16 + m;
                atomicAdd(&dW[((size_t)t * COUT + co) * CIN + ci], acc[a][b][j]);
            }
}

// --------------------------------------------------------------- elementwise

// Network input: channel 0 = r * scale (scale = 1 / rms(r)), channel 1 =
// normalised log kappa (or 0), channels 2..15 = 0; voxels outside n^3 = 0.
// Written as a 16-channel tensor for training (the weight gradient of the
// first layer reads it); inference forms it inside k_conv_in2.
static __global__ void __launch_bounds__(kCB) k_pack_input(const Ctl* __restrict__ ctl, const double* __restrict__ r,
                                                    const double* __restrict__ scale, const bf16* __restrict__ lk,
                                                    bf16* __restrict__ X, int n, int S) {
    if (ctl && ctl->state != 0) return;
    const int v = blockIdx.x * kCB + threadIdx.x;
    if (v >= S * S * S) return;
    const int x = v % S, y = (v / S) % S, z = v / (S * S);
    const bool in = x < n && y < n && z < n;
    const int idx = x + n * (y + n * z);
    const float s = (float)(*scale);
    const bf16 c0 = in ? f2bf((float)r[idx] * s) : (bf16)0;
    const bf16 c1 = (in && lk) ? lk[idx] : (bf16)0;
    const unsigned c01 = (unsigned)c0 | ((unsigned)c1 << 16);
    // all 16 channels (32 bytes) in two 16-byte stores
    uint4* o = reinterpret_cast<uint4*>(X + (size_t)v * 16);
    o[0] = make_uint4(c01, 0u, 0u, 0u);
    o[1] = make_uint4(0u, 0u, 0u, 0u);
}

// Sum of squares of v (N values): per-block partials part[b], fixed order
// (each thread adds its values i, i + stride, ... in increasing i; the loads
// of 8 of them are issued before the additions).
static __global__ void __launch_bounds__(kCB) k_sumsq(const Ctl* __restrict__ ctl, const double* __restrict__ v, int N,
                                               double* __restrict__ part) {
    if (ctl && ctl->state != 0) return;
    constexpr int U = 8;
    const int stride = gridDim.x * kCB;
    double s[1] = {0.0};
    for (int i0 = blockIdx.x * kCB + threadIdx.x; i0 < N; i0 += U * stride) {
        double t[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int i = i0 + j * stride;
            t[j] = i < N ? v[i] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < U; ++j) s[0] += t[j] * t[j];
    }
    block_sum_store<1>(s, part, gridDim.x, blockIdx.x);
}

// mode 0: out = 1 / rms (1 if the values are all zero), rms^2 = sum / N;
// mode 1: out = sum of the partials (the loss).
static __global__ void __launch_bounds__(kRedBlock) k_finish_sum(const Ctl* __restrict__ ctl,
                                                         const double* __restrict__ part, int nblk, int N, int mode,
                                                         double* __restrict__ out) {
    if (ctl && ctl->state != 0) return;
    __shared__ double res[1];
    reduce_partials<1>(part, nblk, res);
    if (threadIdx.x == 0) {
        if (mode == 0) {
            const double rms = sqrt(res[0] / N);
            *out = rms > 0.0 ? 1.0 / rms : 1.0;
        } else {
            *out = res[0];
        }
    }
}

// Y (S^3, C1 + C2 channels) = [upsample2(A) (C1 channels, grid S/2) | B (C2)].
static __global__ void __launch_bounds__(kCB) k_upcat(const Ctl* __restrict__ ctl, const bf16* __restrict__ A,
                                               const bf16* __restrict__ B, bf16* __restrict__ Y, int S, int C1,
                                               int C2) {
    if (ctl && ctl->state != 0) return;
    const int C = C1 + C2;
    const size_t e = (size_t)blockIdx.x * kCB + threadIdx.x;
    if (e >= (size_t)S * S * S * C) return;
    const int c = e % C;
    const size_t v = e / C;
    if (c < C1) {
        const int x = v % S, y = (v / S) % S, z = v / ((size_t)S * S);
        const int Sc = S / 2;
        Y[e] = A[(((size_t)(z / 2) * Sc + y / 2) * Sc + x / 2) * C1 + c];
    } else {
        Y[e] = B[v * C2 + (c - C1)];
    }
}

// dPre = dPost * (post > 0)
static __global__ void __launch_bounds__(kCB) k_relu_mask(const Ctl* __restrict__ ctl, const bf16* __restrict__ dpost,
                                                   const bf16* __restrict__ post, bf16* __restrict__ dpre,
                                                   size_t count) {
    if (ctl && ctl->state != 0) return;
    const size_t e = (size_t)blockIdx.x * kCB + threadIdx.x;
    if (e >= count) return;
    dpre[e] = (bf2f(post[e]) > 0.f) ? dpost[e] : (bf16)0;
}

// dA (S/2 grid, C1 channels) = sum over the 8 children of dY[:, c0 + c]
// (adjoint of nearest upsampling on the first C1 of C channels).
static __global__ void __launch_bounds__(kCB) k_upsample_bwd(const Ctl* __restrict__ ctl, const bf16* __restrict__ dY,
                                                      bf16* __restrict__ dA, int Sc, int C1, int C) {
    if (ctl && ctl->state != 0) return;
    const size_t e = (size_t)blockIdx.x * kCB + threadIdx.x;
    if (e >= (size_t)Sc * Sc * Sc * C1) return;
    const int c = e % C1;
    const size_t v = e / C1;
    const int x = v % Sc, y = (v / Sc) % Sc, z = v / ((size_t)Sc * Sc);
    const int Sf = 2 * Sc;
    float s = 0.f;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int d = 0; d < 2; ++d)
                s += bf2f(dY[(((size_t)(2 * z + a) * Sf + 2 * y + b) * Sf + 2 * x + d) * C + c]);
    dA[e] = f2bf(s);
}

// dE (S^3, C2 channels) = dY[:, C1 + c] (skip part of a concat gradient)
// + upsample2(dP) / 8 (adjoint of average pooling).
static __global__ void __launch_bounds__(kCB) k_skip_pool_bwd(const Ctl* __restrict__ ctl, const bf16* __restrict__ dY,
                                                       const bf16* __restrict__ dP, bf16* __restrict__ dE, int S,
                                                       int C1, int C2) {
    if (ctl && ctl->state != 0) return;
    const size_t e = (size_t)blockIdx.x * kCB + threadIdx.x;
    if (e >= (size_t)S * S * S * C2) return;
    const int c = e % C2;
    const size_t v = e / C2;
    const int x = v % S, y = (v / S) % S, z = v / ((size_t)S * S);
    const int Sc = S / 2;
    const float a = bf2f(dY[v * (C1 + C2) + C1 + c]);
    const float p = bf2f(dP[(((size_t)(z / 2) * Sc + y / 2) * Sc + x / 2) * C2 + c]) * 0.125f;
    dE[e] = f2bf(a + p);
}

// MSE loss over the n^3 voxels against target e * escale; writes the FP32
// loss partials and the bfloat16 gradient (16 channels, channel 0).
static __global__ void __launch_bounds__(kCB) k_mse_grad(const float* __restrict__ out, const double* __restrict__ e,
                                                  const double* __restrict__ escale, bf16* __restrict__ G, int n,
                                                  int S, double* __restrict__ part) {
    const int v = blockIdx.x * kCB + threadIdx.x;
    double l = 0.0;
    if (v < S * S * S) {
        const int x = v % S, y = (v / S) % S, z = v / (S * S);
        const bool in = x < n && y < n && z < n;
        float g = 0.f;
        if (in) {
            const double diff = (double)out[v] - e[x + n * (y + n * z)] * (*escale);
            const double cnt = (double)n * n * n;
            l = diff * diff / cnt;
            g = (float)(2.0 * diff / cnt);
        }
        bf16* o = G + (size_t)v * 16;
        o[0] = f2bf(g);
#pragma unroll
        for (int c = 1; c < 16; ++c) o[c] = 0;
    }
    double acc[1] = {l};
    block_sum_store<1>(acc, part, gridDim.x, blockIdx.x);
}

// Energy loss of the direction d (the network output on the n^3 nodes) for
// the pair (r, e) with q = A d: partial sums of d.r, d.q and e.r.
static __global__ void __launch_bounds__(kCB) k_dots3(const double* __restrict__ d, const double* __restrict__ q,
                                               const double* __restrict__ r, const double* __restrict__ e, int N,
                                               double* __restrict__ part) {
    double v[3] = {0.0, 0.0, 0.0};
    for (int i = blockIdx.x * kCB + threadIdx.x; i < N; i += gridDim.x * kCB) {
        const double ri = r[i], di = d[i];
        v[0] += di * ri;
        v[1] += di * q[i];
        v[2] += e[i] * ri;
    }
    block_sum_store<3>(v, part, gridDim.x, blockIdx.x);
}

// s[0..2] = d.r, d.Ad, e.r; s[3] = loss 1 - (d.r)^2 / ((d.Ad)(e.r)) (1 when
// d.Ad or e.r is not positive).
static __global__ void __launch_bounds__(kRedBlock) k_energy_finish(const double* __restrict__ part, int nblk,
                                                            double* __restrict__ s) {
    __shared__ double res[3];
    reduce_partials<3>(part, nblk, res);
    if (threadIdx.x == 0) {
        const double a = res[0], c = res[1], E = res[2];
        s[0] = a;
        s[1] = c;
        s[2] = E;
        s[3] = (c > 0.0 && E > 0.0) ? 1.0 - a * a / (c * E) : 1.0;
    }
}

// Output gradient of the energy loss, dL/dd = 2a/(cE) ((a/c) q - r), as the
// bfloat16 gradient of channel 0 on the S^3 grid (zero outside the n^3 nodes
// and in the other channels).
static __global__ void __launch_bounds__(kCB) k_energy_grad(const double* __restrict__ s, const double* __restrict__ q,
                                                     const double* __restrict__ r, bf16* __restrict__ G, int n,
                                                     int S) {
    const int v = blockIdx.x * kCB + threadIdx.x;
    if (v >= S * S * S) return;
    const double a = s[0], c = s[1], E = s[2];
    const bool ok = c > 0.0 && E > 0.0;
    const int x = v % S, y = (v / S) % S, z = v / (S * S);
    float g = 0.f;
    if (ok && x < n && y < n && z < n) {
        const int idx = x + n * (y + n * z);
        g = (float)((2.0 * a / (c * E)) * ((a / c) * q[idx] - r[idx]));
    }
    bf16* o = G + (size_t)v * 16;
    o[0] = f2bf(g);
#pragma unroll
    for (int k = 1; k < 16; ++k) o[k] = 0;
}

// dL/dd of the energy loss in FP64 on the n^3 nodes (no network).
static __global__ void __launch_bounds__(kCB) k_energy_grad64(const double* __restrict__ s, const double* __restrict__ q,
                                                       const double* __restrict__ r, double* __restrict__ g, int N) {
    const int i = blockIdx.x * kCB + threadIdx.x;
    if (i >= N) return;
    const double a = s[0], c = s[1], E = s[2];
    g[i] = (c > 0.0 && E > 0.0) ? (2.0 * a / (c * E)) * ((a / c) * q[i] - r[i]) : 0.0;
}

// The network output (the FP32 final layer, one value per voxel) as an MPCG column
// (bulk type T, n^3 values); flag = 1 if any value is not finite.
template <typename T>
__global__ void __launch_bounds__(kCB) k_unpack_output(const Ctl* __restrict__ ctl, const float* __restrict__ out,
                                                       T* __restrict__ d, int n, int S, int* __restrict__ flag) {
    if (ctl && ctl->state != 0) return;
    const int idx = blockIdx.x * kCB + threadIdx.x;
    if (idx >= n * n * n) return;
    const int x = idx % n, y = (idx / n) % n, z = idx / (n * n);
    const float v = out[((size_t)z * S + y) * S + x];
    if (!isfinite(v)) atomicOr(flag, 1);
    d[idx] = T(v);
}

static __global__ void k_clear_flag(const Ctl* __restrict__ ctl, int* flag) {
    if (ctl && ctl->state != 0) return;
    if (threadIdx.x == 0) *flag = 0;
}

// Adam on FP32 masters; refreshes the bfloat16 forward copy [t][co][ci] and
// the tap-flipped, transposed copy [26 - t][ci][co] used by the data gradient.
static __global__ void __launch_bounds__(kCB) k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                                              const float* __restrict__ g, bf16* __restrict__ wb,
                                              bf16* __restrict__ wt, int taps, int cout, int cin, float lr,
                                              float b1, float b2, float eps, float c1, float c2) {
    const int e = blockIdx.x * kCB + threadIdx.x;
    if (e >= taps * cout * cin) return;
    const float gi = g[e];
    const float mi = b1 * m[e] + (1.f - b1) * gi;
    const float vi = b2 * v[e] + (1.f - b2) * gi * gi;
    m[e] = mi;
    v[e] = vi;
    const float wi = w[e] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[e] = wi;
    const bf16 h = f2bf(wi);
    wb[e] = h;
    const int ci = e % cin, co = (e / cin) % cout, t = e / (cin * cout);
    wt[((size_t)(taps - 1 - t) * cin + ci) * cout + co] = h;
}

// bfloat16 copies of FP32 weights (forward and flipped-transposed layouts).
static __global__ void __launch_bounds__(kCB) k_weights_bf16(const float* __restrict__ w, bf16* __restrict__ wb,
                                                      bf16* __restrict__ wt, int taps, int cout, int cin) {
    const int e = blockIdx.x * kCB + threadIdx.x;
    if (e >= taps * cout * cin) return;
    const bf16 h = f2bf(w[e]);
    wb[e] = h;
    const int ci = e % cin, co = (e / cin) % cout, t = e / (cin * cout);
    wt[((size_t)(taps - 1 - t) * cin + ci) * cout + co] = h;
}

}  // namespace cnn
}  // namespace amg
