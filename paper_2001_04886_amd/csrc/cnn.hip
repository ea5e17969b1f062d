// cnn.hip -- learned initial guess x0 = CNN(log k, f) for the restarted
// s-step GMRES of Sec. 4 (Alg 4.2 starts each solve from an arbitrary x0; the
// network that proposes it is an extension beyond the paper).
//
// Network: two input channels (log k, f / rms(f)), four dilated 3x3
// convolutions 2 -> 32 -> 32 -> 32 -> 1 with dilations 1, 2, 4, 8, zero
// padding equal to the dilation, ReLU after the first three; x0 = out *
// rms(f) * out_scale.  Loss: mean squared error against x / (rms(f) *
// out_scale); optimiser: Adam.  Parameters are one FP32 vector, layer by
// layer W_l[Cout][Cin][3][3] then b_l[Cout].
//
// Storage: activations and their gradients are bf16, channels-last
// ([B][H][W][32], 64 bytes per point); every sum accumulates in FP32 (the
// loss and the reductions of per-workgroup partials in FP64).
//
// Kernels:
//   * the two 32 -> 32 layers, forward and data-gradient, are implicit GEMMs on
//     v_mfma_f32_16x16x32_bf16: M = 16 output channels, N = 16 points of a
//     row, K = the 32 input channels of one tap, 9 taps accumulated; a wave
//     keeps all its weights in registers and walks rows group by group, the
//     x-shifted taps formed by lane shifts from the neighbouring groups (3
//     loads per group instead of 9);
//   * their weight gradients contract over points: both operands are staged
//     through LDS transposed (channel-major) so a lane reads 8 consecutive
//     points of one channel, and the 9 taps are 9 MFMA accumulators;
//   * the thin first and last layers (2 inputs, 1 output) run on the FP32
//     vector ALUs: they hold 6% of the flops and cannot fill a 16-wide tile.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "../../include/sstep.h"
#include "kernels.hpp"
#include "launch.hpp"

namespace sstep {
namespace cnn {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int CH = 32;
// offsets (floats) of each block in the parameter vector
constexpr int OW1 = 0, OB1 = OW1 + CH * 2 * 9;
constexpr int OW2 = OB1 + CH, OB2 = OW2 + CH * CH * 9;
constexpr int OW3 = OB2 + CH, OB3 = OW3 + CH * CH * 9;
constexpr int OW4 = OB3 + CH, OB4 = OW4 + CH * 9;
constexpr int NPARAM = OB4 + 1;
static_assert(NPARAM == 19393, "parameter count");
constexpr int DIL1 = 1, DIL2 = 2, DIL3 = 4, DIL4 = 8;

constexpr int kMaxConvWG = 512;  // persistent conv grid: about two workgroups per CU
constexpr int kMaxWgradWG = 1024;
constexpr int kMaxThinWG = 2048;

// weight-gradient tile: one row segment of SEG points, dilation <= DMAX
constexpr int SEG = 64;
constexpr int DMAX = 4;
constexpr int GT_LD = SEG + 8;
constexpr int XT_COLS = SEG + 2 * DMAX;
constexpr int XT_LD = XT_COLS + 8;
constexpr int PS32 = CH * CH * 9 + CH;  // partial size of a 32 -> 32 layer
constexpr int PS1 = CH * 2 * 9 + CH;    // first layer
constexpr int PS4 = CH * 9 + 1;         // last layer

__device__ __forceinline__ bool inside(int y, int x, int H, int W) {
    return y >= 0 && y < H && x >= 0 && x < W;
}

// ---------------------------------------------------------------------------
// input preparation
// ---------------------------------------------------------------------------

// rms(f) per sample (one workgroup per sample); an all-zero f gets 1 so the
// normalised input stays finite.
__global__ __launch_bounds__(kThreads) void k_rms(long long hw, const double* __restrict__ f,
                                                  double* __restrict__ frms) {
    __shared__ double lds[4];
    const double* fp = f + (long long)blockIdx.x * hw;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    long long p = threadIdx.x;
    for (; p + 3 * kThreads < hw; p += 4 * kThreads) {
        const double a = fp[p], b = fp[p + kThreads], c = fp[p + 2 * kThreads],
                     d = fp[p + 3 * kThreads];
        s0 += a * a;
        s1 += b * b;
        s2 += c * c;
        s3 += d * d;
    }
    for (; p < hw; p += kThreads) s0 += fp[p] * fp[p];
    double v1[1] = {(s0 + s1) + (s2 + s3)}, o[1];
    block_sum<1>(v1, lds, o);
    if (threadIdx.x == 0) frms[blockIdx.x] = o[0] > 0.0 ? sqrt(o[0] / (double)hw) : 1.0;
}

// a0 = (log k, f / rms(f)) in bf16 pairs; optional target t = x / (rms(f) * scale).
__global__ __launch_bounds__(kThreads) void k_prep(long long npix, long long hw,
                                                   const float* __restrict__ logk,
                                                   const double* __restrict__ f,
                                                   const double* __restrict__ frms,
                                                   const double* __restrict__ x, double scale,
                                                   bf16x2* __restrict__ a0,
                                                   float* __restrict__ t) {
    const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i >= npix) return;
    const double fr = frms[i / hw];
    bf16x2 v;
    v[0] = (bf16)logk[i];
    v[1] = (bf16)(float)(f[i] / fr);
    a0[i] = v;
    if (x) t[i] = (float)(x[i] / (fr * scale));
}

// ---------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------

// layer 1: 2 -> 32, dilation 1, ReLU; one point per thread, FP32 FMAs.
__global__ __launch_bounds__(kThreads) void k_conv_in(int B, int H, int W,
                                                      const bf16x2* __restrict__ a0,
                                                      const float* __restrict__ prm,
                                                      bf16* __restrict__ a1) {
    // uniform weights: scalar loads (each output channel's 18 are contiguous)
    const float* __restrict__ w = prm + OW1;
    const long long npix = (long long)B * H * W;
    const long long pix = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (pix >= npix) return;
    const int x = (int)(pix % W);
    const int y = (int)((pix / W) % H);
    const long long rowb = pix - x - (long long)y * W;  // first point of the sample
    float in[9][2];
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
        const int yy = y + (tap / 3 - 1) * DIL1, xx = x + (tap % 3 - 1) * DIL1;
        if (inside(yy, xx, H, W)) {
            const bf16x2 v = a0[rowb + (long long)yy * W + xx];
            in[tap][0] = (float)v[0];
            in[tap][1] = (float)v[1];
        } else {
            in[tap][0] = in[tap][1] = 0.f;
        }
    }
    bf16x8 o[4];
#pragma unroll
    for (int co = 0; co < CH; ++co) {
        float acc = w[CH * 18 + co];
#pragma unroll
        for (int ci = 0; ci < 2; ++ci)
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) acc += w[(co * 2 + ci) * 9 + tap] * in[tap][ci];
        o[co / 8][co % 8] = (bf16)fmaxf(acc, 0.f);
    }
    bf16x8* dst = reinterpret_cast<bf16x8*>(a1 + pix * CH);
#pragma unroll
    for (int q = 0; q < 4; ++q) dst[q] = o[q];
}

// Value of the same 32-bit register D lanes to the left / right within each
// row of 16 lanes (lanes without a source in the row: don't care, the caller
// selects another source for them).
template <int D>
__device__ __forceinline__ bf16x8 row_from_left(bf16x8 v) {
    uint4 u = __builtin_bit_cast(uint4, v);
    u.x = __builtin_amdgcn_update_dpp(u.x, u.x, 0x110 + D, 0xf, 0xf, false);
    u.y = __builtin_amdgcn_update_dpp(u.y, u.y, 0x110 + D, 0xf, 0xf, false);
    u.z = __builtin_amdgcn_update_dpp(u.z, u.z, 0x110 + D, 0xf, 0xf, false);
    u.w = __builtin_amdgcn_update_dpp(u.w, u.w, 0x110 + D, 0xf, 0xf, false);
    return __builtin_bit_cast(bf16x8, u);
}
template <int D>
__device__ __forceinline__ bf16x8 row_from_right(bf16x8 v) {
    uint4 u = __builtin_bit_cast(uint4, v);
    u.x = __builtin_amdgcn_update_dpp(u.x, u.x, 0x100 + D, 0xf, 0xf, false);
    u.y = __builtin_amdgcn_update_dpp(u.y, u.y, 0x100 + D, 0xf, 0xf, false);
    u.z = __builtin_amdgcn_update_dpp(u.z, u.z, 0x100 + D, 0xf, 0xf, false);
    u.w = __builtin_amdgcn_update_dpp(u.w, u.w, 0x100 + D, 0xf, 0xf, false);
    return __builtin_bit_cast(bf16x8, u);
}
__device__ __forceinline__ bf16x8 sel8(bool c, bf16x8 a, bf16x8 b) {
    const uint4 ua = __builtin_bit_cast(uint4, a), ub = __builtin_bit_cast(uint4, b);
    uint4 r;
    r.x = c ? ua.x : ub.x;
    r.y = c ? ua.y : ub.y;
    r.z = c ? ua.z : ub.z;
    r.w = c ? ua.w : ub.w;
    return __builtin_bit_cast(bf16x8, r);
}

// 32 -> 32 dilated 3x3 layer on MFMA, dilation D.
//   forward  (DGRAD = false): Y[p][co] = relu(b[co] + sum_{tap,ci} W[co][ci][tap] X[p+off(tap)][ci])
//   data gradient (DGRAD = true):
//            Y[p][ci] = [mask[p][ci] > 0] * sum_{tap,co} W[co][ci][8-tap] X[p+off(tap)][co]
//   (off(8 - tap) = -off(tap), so the adjoint is the same gather with the
//   weights transposed and the taps reversed).
// One wave computes 16 consecutive points of a row x 32 output channels per
// step as two 16x16 MFMA tiles over 9 taps x 32 input channels: lane l holds
// point l mod 16 of the group and input channels 8 (l / 16) .. +8.  The grid
// is persistent (about two workgroups per CU): a workgroup stages the
// layer's weights once, as bf16 in the MFMA lane order, through LDS; each
// wave then walks whole rows group by group.  Of the nine operands of a
// group only the three centre loads (one per tap row) are new: a wave keeps
// the previous, current and next group of each tap row in registers and
// forms the x -/+ D taps by shifting within the 16-lane rows (DPP) from the
// current group and its left / right neighbour, so a group costs 3 loads
// instead of 9.  The next-but-one group's loads are in flight while the
// current group's 18 MFMAs run.  Points outside the grid load as zero.
template <bool DGRAD, int D>
__global__ __launch_bounds__(kThreads) void k_conv32(int B, int H, int W,
                                                     const bf16* __restrict__ X,
                                                     const float* __restrict__ prm, int ow, int ob,
                                                     const bf16* __restrict__ mask,
                                                     bf16* __restrict__ Y) {
    static_assert(D >= 1 && D < 16, "taps must stay within a neighbouring group");
    __shared__ __attribute__((aligned(16))) bf16 wl[9 * 2 * 64 * 8];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int m16 = lane & 15, kq = lane >> 4;
    // A operands: row m16 (+16 h) of the output channels, k = kq*8 + e of the
    // input channels, one per tap and half; entry ((tap*2 + h)*64 + lane)*8 + e
    for (int q = threadIdx.x; q < 9 * 2 * 64 * 8; q += kThreads) {
        const int e = q & 7, l = (q >> 3) & 63, th = q >> 9;
        const int tap = th >> 1, h = th & 1;
        const int mo = h * 16 + (l & 15), ki = (l >> 4) * 8 + e;
        const float v = DGRAD ? prm[ow + (ki * CH + mo) * 9 + (8 - tap)]
                              : prm[ow + (mo * CH + ki) * 9 + tap];
        wl[q] = (bf16)v;
    }
    __syncthreads();
    bf16x8 wa[9][2];
#pragma unroll
    for (int tap = 0; tap < 9; ++tap)
#pragma unroll
        for (int h = 0; h < 2; ++h)
            wa[tap][h] = *reinterpret_cast<const bf16x8*>(wl + ((tap * 2 + h) * 64 + lane) * 8);
    float bias[2][4];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int e = 0; e < 4; ++e) bias[h][e] = DGRAD ? 0.f : prm[ob + h * 16 + kq * 4 + e];

    const int gpr = (W + 15) / 16;
    const long long nrows = (long long)B * H;
    const long long nwaves = (long long)gridDim.x * 4;
    bf16x8 zero8;
#pragma unroll
    for (int e = 0; e < 8; ++e) zero8[e] = (bf16)0.f;
    // the 16-byte load of point px of input row yy (zero outside the grid)
    auto load = [&](long long sbase, int yy, int px) {
        bf16x8 v = zero8;
        if (inside(yy, px, H, W))
            v = *reinterpret_cast<const bf16x8*>(X + (sbase + (long long)yy * W + px) * CH + kq * 8);
        return v;
    };
    for (long long row = (long long)xcd_remap(blockIdx.x, gridDim.x) * 4 + wv; row < nrows;
         row += nwaves) {
        const int y = (int)(row % H);
        const long long sbase = (row - y) * W;
        // tap row r (dy = r - 1): previous, current and next group
        bf16x8 P[3], C[3], N[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            P[r] = zero8;
            C[r] = load(sbase, y + (r - 1) * D, m16);
            N[r] = load(sbase, y + (r - 1) * D, 16 + m16);
        }
        for (int gx = 0; gx < gpr; ++gx) {
            bf16x8 NN[3];
#pragma unroll
            for (int r = 0; r < 3; ++r) NN[r] = load(sbase, y + (r - 1) * D, (gx + 2) * 16 + m16);
            f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                // x - D: this group's lane m16 - D, or the previous group's lane m16 - D + 16
                const bf16x8 bl = sel8(m16 >= D, row_from_left<D>(C[r]), row_from_right<16 - D>(P[r]));
                // x + D: this group's lane m16 + D, or the next group's lane m16 + D - 16
                const bf16x8 br = sel8(m16 + D < 16, row_from_right<D>(C[r]), row_from_left<16 - D>(N[r]));
                acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[r * 3 + 0][0], bl, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[r * 3 + 0][1], bl, acc1, 0, 0, 0);
                acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[r * 3 + 1][0], C[r], acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[r * 3 + 1][1], C[r], acc1, 0, 0, 0);
                acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[r * 3 + 2][0], br, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[r * 3 + 2][1], br, acc1, 0, 0, 0);
            }
            const int px = gx * 16 + m16;
            if (px < W) {
                const long long o = (sbase + (long long)y * W + px) * CH;
                bf16x4 r0, r1;
                if (DGRAD) {
                    const bf16x4 m0 = *reinterpret_cast<const bf16x4*>(mask + o + kq * 4);
                    const bf16x4 m1 = *reinterpret_cast<const bf16x4*>(mask + o + 16 + kq * 4);
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        r0[e] = (bf16)((float)m0[e] > 0.f ? acc0[e] : 0.f);
                        r1[e] = (bf16)((float)m1[e] > 0.f ? acc1[e] : 0.f);
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        r0[e] = (bf16)fmaxf(acc0[e] + bias[0][e], 0.f);
                        r1[e] = (bf16)fmaxf(acc1[e] + bias[1][e], 0.f);
                    }
                }
                *reinterpret_cast<bf16x4*>(Y + o + kq * 4) = r0;
                *reinterpret_cast<bf16x4*>(Y + o + 16 + kq * 4) = r1;
            }
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                P[r] = C[r];
                C[r] = N[r];
                N[r] = NN[r];
            }
        }
    }
}

// layer 4: 32 -> 1, dilation 8, no activation; one point per thread.  Writes
// the raw output and/or the scaled guess x0 = out * rms(f) * scale.
__global__ __launch_bounds__(kThreads) void k_conv_out(int B, int H, int W,
                                                       const bf16* __restrict__ a3,
                                                       const float* __restrict__ prm,
                                                       float* __restrict__ out,
                                                       const double* __restrict__ frms,
                                                       double scale, double* __restrict__ x0) {
    // the weights are uniform across the workgroup: scalar loads, one tap's
    // 32 at a time, feed the FMAs as scalar operands
    const float* __restrict__ w = prm + OW4;
    const long long hw = (long long)H * W, npix = B * hw;
    const long long pix = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (pix >= npix) return;
    const int x = (int)(pix % W);
    const int y = (int)((pix / W) % H);
    const long long sbase = pix - x - (long long)y * W;
    float acc = w[CH * 9];
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
        const int yy = y + (tap / 3 - 1) * DIL4, xx = x + (tap % 3 - 1) * DIL4;
        if (!inside(yy, xx, H, W)) continue;
        const bf16x8* src = reinterpret_cast<const bf16x8*>(a3 + (sbase + (long long)yy * W + xx) * CH);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const bf16x8 v = src[q];
#pragma unroll
            for (int e = 0; e < 8; ++e) acc += w[(q * 8 + e) * 9 + tap] * (float)v[e];
        }
    }
    if (out) out[pix] = acc;
    if (x0) x0[pix] = (double)acc * frms[pix / hw] * scale;
}

// ---------------------------------------------------------------------------
// loss and backward
// ---------------------------------------------------------------------------

// g4 = 2 (out - t) / npix; per-workgroup partial sums of (out - t)^2.
__global__ __launch_bounds__(kThreads) void k_loss(long long npix, const float* __restrict__ out,
                                                   const float* __restrict__ t,
                                                   float* __restrict__ g4,
                                                   double* __restrict__ part) {
    __shared__ double lds[4];
    const float sc = (float)(2.0 / (double)npix);
    double s = 0.0;
    for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < npix;
         i += (long long)gridDim.x * kThreads) {
        const float e = out[i] - t[i];
        g4[i] = sc * e;
        s += (double)e * (double)e;
    }
    double v1[1] = {s}, o[1];
    block_sum<1>(v1, lds, o);
    if (threadIdx.x == 0) part[blockIdx.x] = o[0];
}

// layer 4 data gradient: g3[p][ci] = [a3[p][ci] > 0] * sum_tap W4[ci][tap] g4[p - off(tap)].
__global__ __launch_bounds__(kThreads) void k_dgrad_out(int B, int H, int W,
                                                        const float* __restrict__ g4,
                                                        const float* __restrict__ prm,
                                                        const bf16* __restrict__ a3,
                                                        bf16* __restrict__ g3) {
    __shared__ float w[CH * 9];
    for (int i = threadIdx.x; i < CH * 9; i += kThreads) w[i] = prm[OW4 + i];
    __syncthreads();
    const long long npix = (long long)B * H * W;
    const long long pix = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (pix >= npix) return;
    const int x = (int)(pix % W);
    const int y = (int)((pix / W) % H);
    const long long sbase = pix - x - (long long)y * W;
    float gv[9];
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
        const int yy = y - (tap / 3 - 1) * DIL4, xx = x - (tap % 3 - 1) * DIL4;
        gv[tap] = inside(yy, xx, H, W) ? g4[sbase + (long long)yy * W + xx] : 0.f;
    }
    const bf16x8* m = reinterpret_cast<const bf16x8*>(a3 + pix * CH);
    bf16x8* dst = reinterpret_cast<bf16x8*>(g3 + pix * CH);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const bf16x8 mv = m[q];
        bf16x8 o;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            float acc = 0.f;
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) acc += w[(q * 8 + e) * 9 + tap] * gv[tap];
            o[e] = (bf16)((float)mv[e] > 0.f ? acc : 0.f);
        }
        dst[q] = o;
    }
}

// Grid coordinates (x, y) of the points p0 + g, p0 + g + step, ... advanced
// without divisions (the sample index is not needed: offsets stay in-sample).
struct PixWalk {
    int x, y, W, H;
    long long sbase;  // first point of the current sample
    __device__ PixWalk(long long p, int W_, int H_) : W(W_), H(H_) {
        const long long hw = (long long)W_ * H_;
        sbase = p - p % hw;
        const int r = (int)(p - sbase);
        y = r / W_;
        x = r - y * W_;
    }
    __device__ __forceinline__ void advance(int step) {
        x += step;
        while (x >= W) {
            x -= W;
            if (++y == H) {
                y = 0;
                sbase += (long long)W * H;
            }
        }
    }
};

// Thin-layer weight gradients: thread (pg, task) with task = tap * 4 + cq
// (cq: a chunk of 8 channels, one 16-byte load), pg = 0..6 a point group
// (points p0 + pg, p0 + pg + 7, ... of the workgroup's chunk); the point
// groups are summed through LDS in order.
constexpr int TG_TASKS = 36, TG_GROUPS = kThreads / TG_TASKS;  // 7 groups (252 threads)

// layer 4: dW4[ci][tap] = sum_p g4[p] a3[p + off(tap)][ci], db4 = sum_p g4[p].
__global__ __launch_bounds__(kThreads) void k_wgrad_out(int B, int H, int W, long long chunk,
                                                        const float* __restrict__ g4,
                                                        const bf16* __restrict__ a3,
                                                        float* __restrict__ part) {
    __shared__ float red[TG_GROUPS][PS4 + 3];
    const int task = threadIdx.x % TG_TASKS, pg = threadIdx.x / TG_TASKS;
    const int tap = task >> 2, cq = task & 3;
    const int dy = (tap / 3 - 1) * DIL4, dx = (tap % 3 - 1) * DIL4;
    const long long npix = (long long)B * H * W;
    const long long p0 = (long long)blockIdx.x * chunk;
    const long long p1 = p0 + chunk < npix ? p0 + chunk : npix;
    float acc[8], bacc = 0.f;
#pragma unroll
    for (int e = 0; e < 8; ++e) acc[e] = 0.f;
    if (pg < TG_GROUPS && p0 + pg < p1) {
        PixWalk w(p0 + pg, W, H);
        for (long long p = p0 + pg; p < p1; p += TG_GROUPS, w.advance(TG_GROUPS)) {
            const float g = g4[p];
            if (task == 0) bacc += g;
            const int yy = w.y + dy, xx = w.x + dx;
            if (inside(yy, xx, H, W)) {
                const bf16x8 v = *reinterpret_cast<const bf16x8*>(
                    a3 + (w.sbase + (long long)yy * W + xx) * CH + cq * 8);
#pragma unroll
                for (int e = 0; e < 8; ++e) acc[e] += g * (float)v[e];
            }
        }
    }
    if (pg < TG_GROUPS) {
#pragma unroll
        for (int e = 0; e < 8; ++e) red[pg][(cq * 8 + e) * 9 + tap] = acc[e];
        if (task == 0) red[pg][CH * 9] = bacc;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < PS4; i += kThreads) {
        float t = 0.f;
#pragma unroll
        for (int q = 0; q < TG_GROUPS; ++q) t += red[q][i];
        part[(long long)blockIdx.x * PS4 + i] = t;
    }
}

// weight gradient of a 32 -> 32 layer:
//   dW[co][ci][tap] = sum_p G[p][co] X[p + off(tap)][ci],  db[co] = sum_p G[p][co]
// A unit is one row segment of SEG points.  G's segment and the three rows of
// X it reaches (with DMAX halo columns) are staged in LDS channel-major, so an
// MFMA operand is 8 consecutive points of one channel.  Wave w owns output
// channels 16 (w & 1) .. +15 and input channels 16 (w >> 1) .. +15, 9 taps.
__global__ __launch_bounds__(kThreads) void k_wgrad32(int B, int H, int W, int d,
                                                      const bf16* __restrict__ G,
                                                      const bf16* __restrict__ X,
                                                      float* __restrict__ part) {
    __shared__ __attribute__((aligned(16))) bf16 gT[CH * GT_LD];
    __shared__ __attribute__((aligned(16))) bf16 xT[3 * CH * XT_LD];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m16 = lane & 15, kq = lane >> 4;
    const int mh = wv & 1, chh = wv >> 1;
    f32x4 acc[9];
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) acc[tap] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bacc = 0.f;
    const int segs = (W + SEG - 1) / SEG;
    const long long units = (long long)B * H * segs;
    for (long long u = xcd_remap(blockIdx.x, gridDim.x); u < units; u += gridDim.x) {
        const int seg = (int)(u % segs);
        const long long row = u / segs;
        const int y = (int)(row % H);
        const long long sbase = (row - y) * W;
        const int x0 = seg * SEG;
        __syncthreads();  // the previous unit's operands have been read
        {
            const int px = tid >> 2, c = tid & 3, xx = x0 + px;
            bf16x8 v;
            if (xx < W) {
                v = *reinterpret_cast<const bf16x8*>(G + (sbase + (long long)y * W + xx) * CH + c * 8);
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) v[e] = (bf16)0.f;
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) gT[(c * 8 + e) * GT_LD + px] = v[e];
        }
        for (int idx = tid; idx < 3 * XT_COLS * 4; idx += kThreads) {
            const int r = idx / (XT_COLS * 4), rem = idx % (XT_COLS * 4);
            const int k = rem >> 2, c = rem & 3;
            const int yy = y + (r - 1) * d, xx = x0 - DMAX + k;
            bf16x8 v;
            if (inside(yy, xx, H, W)) {
                v = *reinterpret_cast<const bf16x8*>(X + (sbase + (long long)yy * W + xx) * CH + c * 8);
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) v[e] = (bf16)0.f;
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) xT[(r * CH + c * 8 + e) * XT_LD + k] = v[e];
        }
        __syncthreads();
        if (tid < CH)
            for (int k = 0; k < SEG; ++k) bacc += (float)gT[tid * GT_LD + k];
#pragma unroll
        for (int ks = 0; ks < SEG / 32; ++ks) {
            const bf16x8 a =
                *reinterpret_cast<const bf16x8*>(gT + (mh * 16 + m16) * GT_LD + ks * 32 + kq * 8);
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) {
                const int col = ks * 32 + kq * 8 + DMAX + (tap % 3 - 1) * d;  // even: d is even
                const unsigned* src = reinterpret_cast<const unsigned*>(
                    xT + ((tap / 3) * CH + chh * 16 + m16) * XT_LD + col);
                unsigned u4[4] = {src[0], src[1], src[2], src[3]};
                bf16x8 b;
                __builtin_memcpy(&b, u4, 16);
                acc[tap] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[tap], 0, 0, 0);
            }
        }
    }
    float* dst = part + (long long)blockIdx.x * PS32;
#pragma unroll
    for (int tap = 0; tap < 9; ++tap)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int co = mh * 16 + kq * 4 + e, ci = chh * 16 + m16;
            dst[(co * CH + ci) * 9 + tap] = acc[tap][e];
        }
    if (tid < CH) dst[CH * CH * 9 + tid] = bacc;
}

// layer 1: dW1[co][cin][tap] = sum_p g1[p][co] a0[p + off(tap)][cin],
// db1[co] = sum_p g1[p][co]; cq chunks the output channels co.
__global__ __launch_bounds__(kThreads) void k_wgrad_in(int B, int H, int W, long long chunk,
                                                       const bf16* __restrict__ g1,
                                                       const bf16x2* __restrict__ a0,
                                                       float* __restrict__ part) {
    __shared__ float red[TG_GROUPS][PS1 + 1];
    const int task = threadIdx.x % TG_TASKS, pg = threadIdx.x / TG_TASKS;
    const int tap = task >> 2, cq = task & 3;
    const int dy = (tap / 3 - 1) * DIL1, dx = (tap % 3 - 1) * DIL1;
    const long long npix = (long long)B * H * W;
    const long long p0 = (long long)blockIdx.x * chunk;
    const long long p1 = p0 + chunk < npix ? p0 + chunk : npix;
    float acc[8][2], bacc[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) acc[e][0] = acc[e][1] = bacc[e] = 0.f;
    if (pg < TG_GROUPS && p0 + pg < p1) {
        PixWalk w(p0 + pg, W, H);
        for (long long p = p0 + pg; p < p1; p += TG_GROUPS, w.advance(TG_GROUPS)) {
            const bf16x8 gv = *reinterpret_cast<const bf16x8*>(g1 + p * CH + cq * 8);
            if (tap == 0) {
#pragma unroll
                for (int e = 0; e < 8; ++e) bacc[e] += (float)gv[e];
            }
            const int yy = w.y + dy, xx = w.x + dx;
            if (inside(yy, xx, H, W)) {
                const bf16x2 v = a0[w.sbase + (long long)yy * W + xx];
                const float v0 = (float)v[0], v1 = (float)v[1];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    acc[e][0] += (float)gv[e] * v0;
                    acc[e][1] += (float)gv[e] * v1;
                }
            }
        }
    }
    if (pg < TG_GROUPS) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int co = cq * 8 + e;
            red[pg][(co * 2 + 0) * 9 + tap] = acc[e][0];
            red[pg][(co * 2 + 1) * 9 + tap] = acc[e][1];
            if (tap == 0) red[pg][CH * 18 + co] = bacc[e];
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < PS1; i += kThreads) {
        float t = 0.f;
#pragma unroll
        for (int q = 0; q < TG_GROUPS; ++q) t += red[q][i];
        part[(long long)blockIdx.x * PS1 + i] = t;
    }
}

// grad[i] = sum over parts of part[q][i] (FP64): 8 outputs per workgroup; the
// parts are cut into 32 consecutive ranges, each summed in order by one thread
// (two interleaved accumulators), and the 32 range sums added in order.
constexpr int RP_OUT = 8, RP_GRP = kThreads / RP_OUT;
__global__ __launch_bounds__(kThreads) void k_reduce_parts(const float* __restrict__ part,
                                                           int npart, int psize,
                                                           float* __restrict__ grad) {
    __shared__ double lds[RP_GRP][RP_OUT];
    const int lo = threadIdx.x % RP_OUT, g = threadIdx.x / RP_OUT;
    const int i = blockIdx.x * RP_OUT + lo;
    double s0 = 0.0, s1 = 0.0;
    if (i < psize) {
        const int per = (npart + RP_GRP - 1) / RP_GRP;
        const int q0 = g * per, q1 = min(npart, q0 + per);
        int q = q0;
        for (; q + 1 < q1; q += 2) {
            s0 += (double)part[(long long)q * psize + i];
            s1 += (double)part[(long long)(q + 1) * psize + i];
        }
        if (q < q1) s0 += (double)part[(long long)q * psize + i];
    }
    lds[g][lo] = s0 + s1;
    __syncthreads();
    if (g == 0 && i < psize) {
        double t = 0.0;
        for (int r = 0; r < RP_GRP; ++r) t += lds[r][lo];
        grad[i] = (float)t;
    }
}

// loss = sum of partials / npix (one workgroup)
__global__ __launch_bounds__(kThreads) void k_reduce_loss(const double* __restrict__ part, int n,
                                                          double inv_npix,
                                                          double* __restrict__ loss) {
    __shared__ double lds[4];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += kThreads) s += part[i];
    double v1[1] = {s}, o[1];
    block_sum<1>(v1, lds, o);
    if (threadIdx.x == 0) *loss = o[0] * inv_npix;
}

// Adam with bias-corrected moments; c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t).
// 1 - beta is passed separately (formed in FP64 on the host): 1 - 0.999f in
// FP32 would be off by 1.3e-5 relative.
__global__ __launch_bounds__(kThreads) void k_adam(int n, float* __restrict__ p,
                                                   float* __restrict__ m, float* __restrict__ v,
                                                   const float* __restrict__ g, float lr,
                                                   float b1, float omb1, float b2, float omb2,
                                                   float eps, float c1, float c2) {
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + omb1 * gi;
    const float vi = b2 * v[i] + omb2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// fallback: if ||f - A x0|| >= ||f|| (sums of per-block partials, summed in
// order by one thread), x0 := 0
__global__ void k_fallback_decide(const double* __restrict__ rpart, int nr,
                                  const double* __restrict__ fpart, int nf,
                                  int* __restrict__ flag) {
    if (threadIdx.x != 0) return;
    double a = 0.0, b = 0.0;
    for (int i = 0; i < nr; ++i) a += rpart[i];
    for (int i = 0; i < nf; ++i) b += fpart[i];
    *flag = (a >= b) ? 1 : 0;
}

__global__ __launch_bounds__(kThreads) void k_fallback_apply(long long n, const int* __restrict__ flag,
                                                             double* __restrict__ x0) {
    if (*flag == 0) return;
    for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (long long)gridDim.x * kThreads)
        x0[i] = 0.0;
}

// ---------------------------------------------------------------------------
// coarse-grid guess: block averages, bilinear upsampling, damped Jacobi
// ---------------------------------------------------------------------------

// out[b][J][I] = mean of the fac x fac block of in[b] whose corner is
// (fac J, fac I); sums in FP64, rows of the block in order.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_pool(long long nout, int nx, int nxc, int nyc, int fac,
                                                   const T* __restrict__ in, T* __restrict__ out) {
    const long long hwc = (long long)nxc * nyc;
    for (long long o = (long long)blockIdx.x * kThreads + threadIdx.x; o < nout;
         o += (long long)gridDim.x * kThreads) {
        const long long b = o / hwc, r = o - b * hwc;
        const int J = (int)(r / nxc), I = (int)(r - (long long)J * nxc);
        const T* src = in + b * hwc * fac * fac + ((long long)J * fac) * nx + (long long)I * fac;
        double sum = 0.0;
        for (int jj = 0; jj < fac; ++jj)
            for (int ii = 0; ii < fac; ++ii) sum += (double)src[(long long)jj * nx + ii];
        out[o] = (T)(sum / ((double)fac * fac));
    }
}

// Bilinear interpolation of the coarse field xc [nyc][nxc] (values at the
// centres of the fac x fac blocks) onto the fine grid [ny][nx]: fine point i
// sits at coarse coordinate (i + 1/2)/fac - 1/2; indices outside the coarse
// grid clamp to its edge.
__global__ __launch_bounds__(kThreads) void k_upsample(long long n, int nx, int nxc, int nyc, int fac,
                                                       const double* __restrict__ xc,
                                                       double* __restrict__ x) {
    for (long long p = (long long)blockIdx.x * kThreads + threadIdx.x; p < n;
         p += (long long)gridDim.x * kThreads) {
        const int j = (int)(p / nx), i = (int)(p - (long long)j * nx);
        const double u = (i + 0.5) / fac - 0.5, w = (j + 0.5) / fac - 0.5;
        const double fu = floor(u), fw = floor(w);
        const double tx = u - fu, ty = w - fw;
        const int i0 = (int)fu, j0 = (int)fw;
        const int ia = min(max(i0, 0), nxc - 1), ib = min(max(i0 + 1, 0), nxc - 1);
        const int ja = min(max(j0, 0), nyc - 1), jb = min(max(j0 + 1, 0), nyc - 1);
        const double lo = (1.0 - tx) * xc[(long long)ja * nxc + ia] + tx * xc[(long long)ja * nxc + ib];
        const double hi = (1.0 - tx) * xc[(long long)jb * nxc + ia] + tx * xc[(long long)jb * nxc + ib];
        x[p] = (1.0 - ty) * lo + ty * hi;
    }
}

// One damped Jacobi sweep on the 2-D five-point system:
// xout = xin + omega (f - A xin) / diag(A).
__global__ __launch_bounds__(kThreads) void k_jacobi(StencilView A, const double* __restrict__ f,
                                                     const double* __restrict__ xin,
                                                     double* __restrict__ xout, double omega) {
    const int nx = A.nx, ny = A.ny;
    const long long n = (long long)nx * ny;
    for (long long p = (long long)blockIdx.x * kThreads + threadIdx.x; p < n;
         p += (long long)gridDim.x * kThreads) {
        const int j = (int)(p / nx), i = (int)(p - (long long)j * nx);
        double c[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) c[q] = A.coef ? A.coef[q * A.N + p] : A.c[q];
        double ax = 0.0;
        if (i > 0) ax += c[1] * xin[p - 1];
        if (i < nx - 1) ax += c[2] * xin[p + 1];
        if (j > 0) ax += c[3] * xin[p - nx];
        if (j < ny - 1) ax += c[4] * xin[p + nx];
        ax += c[0] * xin[p];
        xout[p] = xin[p] + omega * (f[p] - ax) / c[0];
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

inline size_t al(size_t b) { return (b + 255) & ~size_t(255); }

inline long long conv_grid(long long groups) {
    const long long wg = (groups + 3) / 4;
    return wg > kMaxConvWG ? kMaxConvWG : (wg < 1 ? 1 : wg);
}
inline long long wgrad_grid(long long units) { return units > kMaxWgradWG ? kMaxWgradWG : units; }
inline long long thin_grid(long long npix) {
    long long wg = (npix + 1023) / 1024;
    return wg > kMaxThinWG ? kMaxThinWG : (wg < 1 ? 1 : wg);
}
inline int loss_grid(long long npix) {
    long long wg = (npix + kThreads - 1) / kThreads;
    return (int)(wg > 1024 ? 1024 : wg);
}

// Workspace regions (byte offsets, 256-byte aligned).  Forward: rms, a0..a3,
// out.  Training adds the target, the gradients, the partials, the parameter
// gradient and the loss.  The fallback test adds the residual and its partials.
struct Layout {
    size_t frms, a0, a1, a2, a3, out;
    size_t t, g4, gA, gB, part, lpart, grad, loss;
    size_t r, rpart, fpart, flag;
    size_t total;
};

inline Layout layout(int B, int H, int W, bool training, bool fallback) {
    const long long npix = (long long)B * H * W;
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += al(bytes);
        return at;
    };
    L.frms = take(8 * (size_t)B);
    L.a0 = take(4 * (size_t)npix);
    L.a1 = take(64 * (size_t)npix);
    L.a2 = take(64 * (size_t)npix);
    L.a3 = take(64 * (size_t)npix);
    L.out = take(4 * (size_t)npix);
    if (training) {
        L.t = take(4 * (size_t)npix);
        L.g4 = take(4 * (size_t)npix);
        L.gA = take(64 * (size_t)npix);
        L.gB = take(64 * (size_t)npix);
        const long long segs = (W + SEG - 1) / SEG;
        size_t pf = (size_t)wgrad_grid((long long)B * H * segs) * PS32;
        const size_t thin = (size_t)thin_grid(npix) * PS1;
        if (thin > pf) pf = thin;
        L.part = take(4 * pf);
        L.lpart = take(8 * (size_t)loss_grid(npix));
        L.grad = take(4 * (size_t)NPARAM);
        L.loss = take(8);
    }
    if (fallback) {
        // residual partials: one per 256-point row segment (2-D grid)
        const long long rblocks = (long long)B * H * ((W + kThreads - 1) / kThreads);
        L.r = take(8 * (size_t)npix);
        L.rpart = take(8 * (size_t)rblocks);
        L.fpart = take(8 * 1024);
        L.flag = take(16);
    }
    L.total = o;
    return L;
}

struct Bufs {
    double* frms;
    bf16x2* a0;
    bf16 *a1, *a2, *a3, *gA, *gB;
    float *out, *t, *g4, *part, *grad;
    double *lpart, *loss, *r, *rpart, *fpart;
    int* flag;
};

inline Bufs bufs(char* ws, const Layout& L, bool training, bool fallback) {
    Bufs b{};
    b.frms = (double*)(ws + L.frms);
    b.a0 = (bf16x2*)(ws + L.a0);
    b.a1 = (bf16*)(ws + L.a1);
    b.a2 = (bf16*)(ws + L.a2);
    b.a3 = (bf16*)(ws + L.a3);
    b.out = (float*)(ws + L.out);
    if (training) {
        b.t = (float*)(ws + L.t);
        b.g4 = (float*)(ws + L.g4);
        b.gA = (bf16*)(ws + L.gA);
        b.gB = (bf16*)(ws + L.gB);
        b.part = (float*)(ws + L.part);
        b.lpart = (double*)(ws + L.lpart);
        b.grad = (float*)(ws + L.grad);
        b.loss = (double*)(ws + L.loss);
    }
    if (fallback) {
        b.r = (double*)(ws + L.r);
        b.rpart = (double*)(ws + L.rpart);
        b.fpart = (double*)(ws + L.fpart);
        b.flag = (int*)(ws + L.flag);
    }
    return b;
}

// Workspace of the coarse-grid guess: the network's forward pass on the
// coarse grid, the pooled inputs and the coarse guess, one fine vector for the
// Jacobi sweeps, and the fine-grid fallback test (residual and partials).
struct CoarseLayout {
    Layout net;  // offsets relative to `net_at`
    size_t net_at, logk_c, f_c, x_c, tmp, r, rpart, fpart, flag, total;
};

inline CoarseLayout coarse_layout(int nx, int ny, int fac) {
    const int nxc = nx / fac, nyc = ny / fac;
    const long long nc = (long long)nxc * nyc, n = (long long)nx * ny;
    CoarseLayout C{};
    C.net = layout(1, nyc, nxc, false, false);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += al(bytes);
        return at;
    };
    C.net_at = take(C.net.total);
    C.logk_c = take(4 * (size_t)nc);
    C.f_c = take(8 * (size_t)nc);
    C.x_c = take(8 * (size_t)nc);
    C.tmp = take(8 * (size_t)n);
    C.r = take(8 * (size_t)n);
    C.rpart = take(8 * (size_t)ny * ((nx + kThreads - 1) / kThreads));
    C.fpart = take(8 * 1024);
    C.flag = take(16);
    C.total = o;
    return C;
}

inline unsigned pix_blocks(long long npix) { return (unsigned)((npix + kThreads - 1) / kThreads); }

// forward pass: a0..a3, out (and x0 if given)
void forward(hipStream_t st, int B, int H, int W, const float* prm, const float* logk,
             const double* f, const double* x, double scale, const Bufs& b, double* x0) {
    const long long hw = (long long)H * W, npix = B * hw;
    hipLaunchKernelGGL(k_rms, dim3(B), dim3(kThreads), 0, st, hw, f, b.frms);
    hipLaunchKernelGGL(k_prep, dim3(pix_blocks(npix)), dim3(kThreads), 0, st, npix, hw, logk, f,
                       (const double*)b.frms, x, scale, b.a0, b.t);
    hipLaunchKernelGGL(k_conv_in, dim3(pix_blocks(npix)), dim3(kThreads), 0, st, B, H, W,
                       (const bf16x2*)b.a0, prm, b.a1);
    const long long groups = (long long)B * H * ((W + 15) / 16);
    const unsigned cg = (unsigned)conv_grid(groups);
    hipLaunchKernelGGL((k_conv32<false, DIL2>), dim3(cg), dim3(kThreads), 0, st, B, H, W,
                       (const bf16*)b.a1, prm, OW2, OB2, (const bf16*)nullptr, b.a2);
    hipLaunchKernelGGL((k_conv32<false, DIL3>), dim3(cg), dim3(kThreads), 0, st, B, H, W,
                       (const bf16*)b.a2, prm, OW3, OB3, (const bf16*)nullptr, b.a3);
    hipLaunchKernelGGL(k_conv_out, dim3(pix_blocks(npix)), dim3(kThreads), 0, st, B, H, W,
                       (const bf16*)b.a3, prm, b.out, (const double*)b.frms, scale, x0);
    SSTEP_HIP(hipGetLastError());
}

// gradient of the loss into b.grad (and the loss into *loss_dev)
void backward(hipStream_t st, int B, int H, int W, const float* prm, const Bufs& b,
              double* loss_dev) {
    const long long npix = (long long)B * H * W;
    const int lg = loss_grid(npix);
    hipLaunchKernelGGL(k_loss, dim3(lg), dim3(kThreads), 0, st, npix, (const float*)b.out,
                       (const float*)b.t, b.g4, b.lpart);
    hipLaunchKernelGGL(k_reduce_loss, dim3(1), dim3(kThreads), 0, st, (const double*)b.lpart, lg,
                       1.0 / (double)npix, loss_dev);
    const unsigned rb = (unsigned)((PS32 + RP_OUT - 1) / RP_OUT);
    // layer 4
    const long long tg = thin_grid(npix), chunk = (npix + tg - 1) / tg;
    hipLaunchKernelGGL(k_wgrad_out, dim3((unsigned)tg), dim3(kThreads), 0, st, B, H, W, chunk,
                       (const float*)b.g4, (const bf16*)b.a3, b.part);
    hipLaunchKernelGGL(k_reduce_parts, dim3(rb), dim3(kThreads), 0, st, (const float*)b.part,
                       (int)tg, PS4, b.grad + OW4);
    hipLaunchKernelGGL(k_dgrad_out, dim3(pix_blocks(npix)), dim3(kThreads), 0, st, B, H, W,
                       (const float*)b.g4, prm, (const bf16*)b.a3, b.gA);
    // layer 3 (gA = dL/dz3) and layer 2 (gB = dL/dz2)
    const long long segs = (W + SEG - 1) / SEG;
    const unsigned wg = (unsigned)wgrad_grid((long long)B * H * segs);
    const long long groups = (long long)B * H * ((W + 15) / 16);
    const unsigned cg = (unsigned)conv_grid(groups);
    hipLaunchKernelGGL(k_wgrad32, dim3(wg), dim3(kThreads), 0, st, B, H, W, DIL3,
                       (const bf16*)b.gA, (const bf16*)b.a2, b.part);
    hipLaunchKernelGGL(k_reduce_parts, dim3(rb), dim3(kThreads), 0, st, (const float*)b.part,
                       (int)wg, PS32, b.grad + OW3);
    hipLaunchKernelGGL((k_conv32<true, DIL3>), dim3(cg), dim3(kThreads), 0, st, B, H, W,
                       (const bf16*)b.gA, prm, OW3, 0, (const bf16*)b.a2, b.gB);
    hipLaunchKernelGGL(k_wgrad32, dim3(wg), dim3(kThreads), 0, st, B, H, W, DIL2,
                       (const bf16*)b.gB, (const bf16*)b.a1, b.part);
    hipLaunchKernelGGL(k_reduce_parts, dim3(rb), dim3(kThreads), 0, st, (const float*)b.part,
                       (int)wg, PS32, b.grad + OW2);
    hipLaunchKernelGGL((k_conv32<true, DIL2>), dim3(cg), dim3(kThreads), 0, st, B, H, W,
                       (const bf16*)b.gB, prm, OW2, 0, (const bf16*)b.a1, b.gA);
    // layer 1 (gA = dL/dz1)
    hipLaunchKernelGGL(k_wgrad_in, dim3((unsigned)tg), dim3(kThreads), 0, st, B, H, W, chunk,
                       (const bf16*)b.gA, (const bf16x2*)b.a0, b.part);
    hipLaunchKernelGGL(k_reduce_parts, dim3(rb), dim3(kThreads), 0, st, (const float*)b.part,
                       (int)tg, PS1, b.grad + OW1);
    SSTEP_HIP(hipGetLastError());
}

void adam(hipStream_t st, float* p, float* m, float* v, const float* g, int step, float lr) {
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = (float)(1.0 / (1.0 - std::pow(b1, step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow(b2, step)));
    hipLaunchKernelGGL(k_adam, dim3((NPARAM + kThreads - 1) / kThreads), dim3(kThreads), 0, st,
                       NPARAM, p, m, v, g, lr, (float)b1, (float)(1.0 - b1), (float)b2,
                       (float)(1.0 - b2), 1e-8f, c1, c2);
    SSTEP_HIP(hipGetLastError());
}

}  // namespace cnn
}  // namespace sstep

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
using namespace sstep;

namespace {

bool al16(const void* p) { return ((uintptr_t)p & 15) == 0; }

bool dims_ok(int B, int nx, int ny) {
    if (B < 1 || nx < 1 || ny < 1) return false;
    const long long npix = (long long)B * nx * ny;
    return npix <= (1LL << 31) - 1;
}

template <typename F>
int cnn_guard(F&& fn) {
    try {
        return fn();
    } catch (const HipFailure&) {
        (void)hipGetLastError();
        return SSTEP_ERR_HIP;
    }
}

// Runs fn(ws) with the caller's workspace or a temporary one; waits for the
// stream before returning.
template <typename F>
int with_workspace(const sstep_options* opt, size_t need, F&& fn) {
    sstep_options o;
    if (opt) o = *opt;
    else sstep_default_options(&o);
    hipStream_t st = (hipStream_t)o.stream;
    return cnn_guard([&]() -> int {
        char* ws = (char*)o.workspace;
        bool owned = false;
        if (ws) {
            if (o.workspace_bytes < need || !al16(ws)) return SSTEP_ERR_ARG;
        } else {
            if (hipMalloc((void**)&ws, need) != hipSuccess) {
                (void)hipGetLastError();
                return SSTEP_ERR_NOMEM;
            }
            owned = true;
        }
        int st_code = SSTEP_OK;
        try {
            st_code = fn(st, ws);
            SSTEP_HIP(hipStreamSynchronize(st));
        } catch (...) {
            if (owned) (void)hipFree(ws);
            throw;
        }
        if (owned) SSTEP_HIP(hipFree(ws));
        return st_code;
    });
}

}  // namespace

extern "C" {

size_t sstep_cnn_param_count(void) { return (size_t)cnn::NPARAM; }

size_t sstep_cnn_workspace_bytes(int batch, int nx, int ny, int training) {
    if (!dims_ok(batch, nx, ny)) return 0;
    // training calls need the training layout; forward and x0_predict (with
    // its fallback test, the larger of the two) the other
    return training ? cnn::layout(batch, ny, nx, true, false).total
                    : cnn::layout(batch, ny, nx, false, true).total;
}

int sstep_cnn_forward(const float* params, double out_scale, int batch, int nx, int ny,
                      const float* logk, const double* f, float* out, double* x0,
                      const sstep_options* opt) {
    if (!dims_ok(batch, nx, ny) || !params || !logk || !f || (!out && !x0)) return SSTEP_ERR_ARG;
    if (!al16(params) || !al16(logk) || !al16(f) || (out && !al16(out)) || (x0 && !al16(x0)) ||
        !(out_scale > 0.0) || !std::isfinite(out_scale))
        return SSTEP_ERR_ARG;
    const cnn::Layout L = cnn::layout(batch, ny, nx, false, false);
    return with_workspace(opt, L.total, [&](hipStream_t st, char* ws) {
        const cnn::Bufs b = cnn::bufs(ws, L, false, false);
        cnn::forward(st, batch, ny, nx, params, logk, f, nullptr, out_scale, b, x0);
        if (out)
            SSTEP_HIP(hipMemcpyAsync(out, b.out, 4 * (size_t)batch * nx * ny,
                                     hipMemcpyDeviceToDevice, st));
        return SSTEP_OK;
    });
}

int sstep_cnn_gradient(const float* params, double out_scale, int batch, int nx, int ny,
                       const float* logk, const double* f, const double* x, float* grad,
                       double* loss, const sstep_options* opt) {
    if (!dims_ok(batch, nx, ny) || !params || !logk || !f || !x || !grad) return SSTEP_ERR_ARG;
    if (!al16(params) || !al16(logk) || !al16(f) || !al16(x) || !al16(grad) ||
        !(out_scale > 0.0) || !std::isfinite(out_scale))
        return SSTEP_ERR_ARG;
    const cnn::Layout L = cnn::layout(batch, ny, nx, true, false);
    return with_workspace(opt, L.total, [&](hipStream_t st, char* ws) {
        const cnn::Bufs b = cnn::bufs(ws, L, true, false);
        cnn::forward(st, batch, ny, nx, params, logk, f, x, out_scale, b, nullptr);
        cnn::backward(st, batch, ny, nx, params, b, b.loss);
        SSTEP_HIP(hipMemcpyAsync(grad, b.grad, 4 * (size_t)cnn::NPARAM, hipMemcpyDeviceToDevice,
                                 st));
        if (loss) SSTEP_HIP(hipMemcpyAsync(loss, b.loss, 8, hipMemcpyDeviceToHost, st));
        return SSTEP_OK;
    });
}

int sstep_cnn_adam(float* params, float* m, float* v, const float* grad, int step, float lr,
                   const sstep_options* opt) {
    if (!params || !m || !v || !grad || step < 1 || !(lr > 0.f) || !std::isfinite(lr))
        return SSTEP_ERR_ARG;
    if (!al16(params) || !al16(m) || !al16(v) || !al16(grad)) return SSTEP_ERR_ARG;
    sstep_options o;
    if (opt) o = *opt;
    else sstep_default_options(&o);
    hipStream_t st = (hipStream_t)o.stream;
    return cnn_guard([&]() -> int {
        cnn::adam(st, params, m, v, grad, step, lr);
        SSTEP_HIP(hipStreamSynchronize(st));
        return SSTEP_OK;
    });
}

int sstep_cnn_train_step(float* params, float* m, float* v, int step, float lr, double out_scale,
                         int batch, int nx, int ny, const float* logk, const double* f,
                         const double* x, double* loss, const sstep_options* opt) {
    if (!dims_ok(batch, nx, ny) || !params || !m || !v || !logk || !f || !x || step < 1 ||
        !(lr > 0.f) || !std::isfinite(lr) || !(out_scale > 0.0) || !std::isfinite(out_scale))
        return SSTEP_ERR_ARG;
    if (!al16(params) || !al16(m) || !al16(v) || !al16(logk) || !al16(f) || !al16(x))
        return SSTEP_ERR_ARG;
    const cnn::Layout L = cnn::layout(batch, ny, nx, true, false);
    return with_workspace(opt, L.total, [&](hipStream_t st, char* ws) {
        const cnn::Bufs b = cnn::bufs(ws, L, true, false);
        cnn::forward(st, batch, ny, nx, params, logk, f, x, out_scale, b, nullptr);
        cnn::backward(st, batch, ny, nx, params, b, b.loss);
        cnn::adam(st, params, m, v, b.grad, step, lr);
        if (loss) SSTEP_HIP(hipMemcpyAsync(loss, b.loss, 8, hipMemcpyDeviceToHost, st));
        return SSTEP_OK;
    });
}

int sstep_x0_predict(const float* params, double out_scale, const sstep_stencil* A,
                     const float* logk, const double* f, double* x0, int use_fallback,
                     int* used_fallback, const sstep_options* opt) {
    if (used_fallback) *used_fallback = 0;
    if (!A || A->ndim != 2 || !dims_ok(1, A->nx, A->ny) || !params || !logk || !f || !x0 ||
        !(out_scale > 0.0) || !std::isfinite(out_scale))
        return SSTEP_ERR_ARG;
    if (!al16(params) || !al16(logk) || !al16(f) || !al16(x0) || (A->coef && !al16(A->coef)))
        return SSTEP_ERR_ARG;
    if (!A->coef)
        for (int q = 0; q < 5; ++q)
            if (!std::isfinite(A->c[q])) return SSTEP_ERR_ARG;
    const int nx = A->nx, ny = A->ny;
    const bool fb = use_fallback != 0;
    const cnn::Layout L = cnn::layout(1, ny, nx, false, fb);
    return with_workspace(opt, L.total, [&](hipStream_t st, char* ws) {
        const cnn::Bufs b = cnn::bufs(ws, L, false, fb);
        cnn::forward(st, 1, ny, nx, params, logk, f, nullptr, out_scale, b, x0);
        if (fb) {
            Ctx c;
            c.st = st;
            const StencilView v = make_view(*A);
            launch_residual<double>(c, v, f, x0, b.r, b.rpart);
            launch_norm2(c, v.N, f, b.fpart);
            hipLaunchKernelGGL(cnn::k_fallback_decide, dim3(1), dim3(64), 0, st,
                               (const double*)b.rpart, (int)stencil_blocks(v),
                               (const double*)b.fpart, norm_blocks(v.N), b.flag);
            hipLaunchKernelGGL(cnn::k_fallback_apply, dim3(norm_blocks(v.N)), dim3(kThreads), 0,
                               st, v.N, (const int*)b.flag, x0);
            SSTEP_HIP(hipGetLastError());
            if (used_fallback)
                SSTEP_HIP(hipMemcpyAsync(used_fallback, b.flag, 4, hipMemcpyDeviceToHost, st));
        }
        return SSTEP_OK;
    });
}

int sstep_grid_pool(const double* in, double* out, int batch, int nx, int ny, int factor,
                    void* stream) {
    if (!in || !out || !dims_ok(batch, nx, ny) || factor < 1 || nx % factor || ny % factor)
        return SSTEP_ERR_ARG;
    return cnn_guard([&]() -> int {
        const hipStream_t st = (hipStream_t)stream;
        const int nxc = nx / factor, nyc = ny / factor;
        const long long nout = (long long)batch * nxc * nyc;
        hipLaunchKernelGGL(cnn::k_pool<double>, dim3(cnn::pix_blocks(nout)), dim3(kThreads), 0, st,
                           nout, nx, nxc, nyc, factor, in, out);
        SSTEP_HIP(hipGetLastError());
        SSTEP_HIP(hipStreamSynchronize(st));
        return SSTEP_OK;
    });
}

size_t sstep_x0_coarse_workspace_bytes(int nx, int ny, int factor) {
    if (!dims_ok(1, nx, ny) || factor < 1 || nx % factor || ny % factor) return 0;
    return cnn::coarse_layout(nx, ny, factor).total;
}

int sstep_x0_predict_coarse(const float* params, double out_scale, int factor, int sweeps,
                            const sstep_stencil* A, const float* logk, const double* f, double* x0,
                            int use_fallback, int* used_fallback, const sstep_options* opt) {
    if (used_fallback) *used_fallback = 0;
    if (!A || A->ndim != 2 || !dims_ok(1, A->nx, A->ny) || !params || !logk || !f || !x0 ||
        !(out_scale > 0.0) || !std::isfinite(out_scale) || factor < 1 || A->nx % factor ||
        A->ny % factor || sweeps < 0 || sweeps > 100000)
        return SSTEP_ERR_ARG;
    if (!al16(params) || !al16(logk) || !al16(f) || !al16(x0) || (A->coef && !al16(A->coef)))
        return SSTEP_ERR_ARG;
    if (!A->coef)
        for (int q = 0; q < 5; ++q)
            if (!std::isfinite(A->c[q])) return SSTEP_ERR_ARG;
    const int nx = A->nx, ny = A->ny, nxc = nx / factor, nyc = ny / factor;
    const long long nc = (long long)nxc * nyc, n = (long long)nx * ny;
    const cnn::CoarseLayout C = cnn::coarse_layout(nx, ny, factor);
    return with_workspace(opt, C.total, [&](hipStream_t st, char* ws) {
        float* logk_c = (float*)(ws + C.logk_c);
        double* f_c = (double*)(ws + C.f_c);
        double* x_c = (double*)(ws + C.x_c);
        double* tmp = (double*)(ws + C.tmp);
        hipLaunchKernelGGL(cnn::k_pool<float>, dim3(cnn::pix_blocks(nc)), dim3(kThreads), 0, st, nc,
                           nx, nxc, nyc, factor, logk, logk_c);
        hipLaunchKernelGGL(cnn::k_pool<double>, dim3(cnn::pix_blocks(nc)), dim3(kThreads), 0, st, nc,
                           nx, nxc, nyc, factor, f, f_c);
        SSTEP_HIP(hipGetLastError());
        const cnn::Bufs b = cnn::bufs(ws + C.net_at, C.net, false, false);
        cnn::forward(st, 1, nyc, nxc, params, logk_c, f_c, nullptr, out_scale, b, x_c);
        hipLaunchKernelGGL(cnn::k_upsample, dim3(cnn::pix_blocks(n)), dim3(kThreads), 0, st, n, nx,
                           nxc, nyc, factor, (const double*)x_c, x0);
        SSTEP_HIP(hipGetLastError());
        const StencilView v = make_view(*A);
        // damped Jacobi sweeps, alternating between x0 and tmp
        constexpr double kOmega = 0.8;
        for (int k = 0; k < sweeps; ++k) {
            const double* src = (k % 2 == 0) ? x0 : tmp;
            double* dst = (k % 2 == 0) ? tmp : x0;
            hipLaunchKernelGGL(cnn::k_jacobi, dim3(cnn::pix_blocks(n)), dim3(kThreads), 0, st, v, f,
                               src, dst, kOmega);
        }
        SSTEP_HIP(hipGetLastError());
        if (sweeps % 2 == 1)
            SSTEP_HIP(hipMemcpyAsync(x0, tmp, 8 * (size_t)n, hipMemcpyDeviceToDevice, st));
        if (use_fallback) {
            Ctx c;
            c.st = st;
            double* r = (double*)(ws + C.r);
            double* rpart = (double*)(ws + C.rpart);
            double* fpart = (double*)(ws + C.fpart);
            int* flag = (int*)(ws + C.flag);
            launch_residual<double>(c, v, f, x0, r, rpart);
            launch_norm2(c, v.N, f, fpart);
            hipLaunchKernelGGL(cnn::k_fallback_decide, dim3(1), dim3(64), 0, st, (const double*)rpart,
                               (int)stencil_blocks(v), (const double*)fpart, norm_blocks(v.N), flag);
            hipLaunchKernelGGL(cnn::k_fallback_apply, dim3(norm_blocks(v.N)), dim3(kThreads), 0, st,
                               v.N, (const int*)flag, x0);
            SSTEP_HIP(hipGetLastError());
            if (used_fallback)
                SSTEP_HIP(hipMemcpyAsync(used_fallback, flag, 4, hipMemcpyDeviceToHost, st));
        }
        return SSTEP_OK;
    });
}

}  // extern "C"
