// The smoothing gate: a small CNN that decides per image whether the hybrid
// median is applied.  The paper leaves that choice to the user, according
// to the noise in the extracted map (abstract; Sec. 4).
//
// Network: three 3x3 convolutions of stride 2 with zero padding
// (3 -> 16 -> 32 -> 32 channels, 128 -> 64 -> 32 -> 16), ReLU after each,
// global average pooling and a linear layer to one logit.  The convolutions
// run as implicit GEMMs on v_mfma_f32_16x16x16_bf16 with FP32 accumulation:
// forward, a workgroup stages its input rows and the weights in LDS; the
// backward kernels gather their operands from the activation maps, one
// wave per 16 x (all channels) block.  Stored activations and their
// gradients are bfloat16; biases, the head, the loss and AdamW are FP32.
// Every reduction has a fixed order (split-K partials are summed in split
// order, no float atomics), so a training step is deterministic.
#include "logfx_gate.h"

namespace logfx {
namespace gate {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline uint16_t to_bf16(float f) {
    // round to nearest, ties to even (finite values)
    const uint32_t u = __float_as_uint(f);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ inline float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// D += A B on one 16 x 16 x 16 block.  Operand layout of the instruction:
// lane l = 16 q + c holds A(c, 4q + i) and B(4q + i, c) for i = 0..3, and
// receives D(4q + i, c).
__device__ inline f32x4 mfma(const bf16x4 &a, const bf16x4 &b, const f32x4 &d) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, d, 0, 0, 0);
}

template <int CI, int CO, int HI>
struct Geo {
    static constexpr int HO = HI / 2, HWI = HI * HI, HWO = HO * HO;
    static constexpr int K = CI * 9, KP = (K + 15) / 16 * 16;   // weights per output channel
    static constexpr int NW1 = K + 1;                            // weight-gradient columns + bias
    static constexpr int NT = (NW1 + 15) / 16;                   // 16-column tiles of them
    static constexpr int MB = CO / 16;
    static_assert(CO % 16 == 0 && HWO % 16 == 0, "layer shape");
};

// ---------------------------------------------------------------- forward
// out[b][co][p] = bf16(relu(bias[co] + sum_{ci,ky,kx} w[co][ci][ky][kx] in[b][ci][2oy+ky-1][2ox+kx-1]))
// for output pixel p = (oy, ox).  GEMM rows = co, columns = 16 pixels of one
// output row, reduction over k = (tap, ci), tap = 3 ky + kx, channels
// padded to a multiple of four (CI = 3 -> 4, with zero weights).
//
// A workgroup takes TH output rows of one image.  It first stages in LDS
// the 2 TH + 1 input rows they read, channel-innermost (one 8-byte slot per
// four channels of a pixel, column -1 and row -1 as the zero padding), and
// copies the layer's weights, kept in that [co][k] order beside the flat
// parameters, as they are; a lane's four reduction indices of a
// 16-deep block are then four consecutive channels at one tap, so each
// MFMA operand is one 8-byte LDS read.  Neighbouring lanes of an operand
// read pixels two apart (an odd number of slots per pixel) or weight rows
// 2 (mod 4) words apart, so the 32 lanes of a half-wave hit distinct banks.  Each of the four waves computes PW
// blocks of 16 pixels for all output channels.
template <int CI, int HI, int TH>
struct Stage {
    static constexpr int CIP = perm_cip(CI);            // padded channels
    static constexpr int G4 = CIP / 4;                  // four-channel groups per pixel
    static constexpr int P = G4 % 2 ? G4 : G4 + 1;      // 8-byte slots per pixel
    static constexpr int X = HI + 1;                    // columns -1 .. HI-1
    static constexpr int R = 2 * TH + 1;                // input rows of TH output rows
    static constexpr int KB = (9 * CIP + 15) / 16;      // 16-deep reduction blocks
    static constexpr int KROW = perm_row(CI);           // weight row: KB * 16 + 8
    static_assert(KROW == KB * 16 + 8, "weight row of the forward layout");
};

template <int CI, int CO, int HI, int TH>
__global__ __launch_bounds__(256) void conv_fwd(const uint16_t *__restrict__ in, const int *__restrict__ idx,
                                                const uint16_t *__restrict__ w, const float *__restrict__ bias,
                                                uint16_t *__restrict__ out, int B) {
    using G = Geo<CI, CO, HI>;
    using S = Stage<CI, HI, TH>;
    constexpr int HO = G::HO, BR = HO / 16, NB = TH * BR, PW = NB / 4, TILES = HO / TH;
    static_assert(HO % TH == 0 && NB % 4 == 0 && HI % 4 == 0, "tile shape");
    typedef uint32_t u32x2a2 __attribute__((ext_vector_type(2), aligned(2)));
    __shared__ uint2 xs[S::R * S::X * S::P];
    __shared__ __align__(16) uint16_t ws[CO * S::KROW];
    const int b = blockIdx.x / TILES, oy0 = (blockIdx.x % TILES) * TH;
    if (b >= B) return;   // uniform over the workgroup
    const int t = threadIdx.x;
    const uint16_t *ib = in + (long long)(idx ? idx[b] : b) * CI * G::HWI;

    // Input rows 2 oy0 - 1 .. 2 oy0 + 2 TH - 1: four pixels of four channels
    // per item, read as one 8-byte word per channel and written as four
    // slots; the weights in 16-byte chunks.  All reads are issued before
    // the first LDS write.
    constexpr int XQ = HI / 4, NI = S::R * S::G4 * XQ, UI = (NI + 255) / 256;
    constexpr int NW = CO * S::KROW / 8, UW = (NW + 255) / 256;
    static_assert((CO * S::KROW) % 8 == 0, "weights in 8-element chunks");
    uint32_t v[UI][4][2];
    uint4 wc[UW];
#pragma unroll
    for (int u = 0; u < UI; ++u) {
        const int it = t + 256 * u, xq = it % XQ, rg = it / XQ, g = rg % S::G4, r = rg / S::G4;
        const int iy = 2 * oy0 - 1 + r;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int ch = 4 * g + j;
            if (it < NI && ch < CI && iy >= 0) {
                const u32x2a2 x = *reinterpret_cast<const u32x2a2 *>(ib + ch * G::HWI + iy * HI + 4 * xq);
                v[u][j][0] = x.x;
                v[u][j][1] = x.y;
            } else {
                v[u][j][0] = v[u][j][1] = 0u;
            }
        }
    }
#pragma unroll
    for (int u = 0; u < UW; ++u) {
        const int it = t + 256 * u;
        wc[u] = it < NW ? reinterpret_cast<const uint4 *>(w)[it] : make_uint4(0u, 0u, 0u, 0u);
    }
#pragma unroll
    for (int u = 0; u < UI; ++u) {
        const int it = t + 256 * u, xq = it % XQ, rg = it / XQ, g = rg % S::G4, r = rg / S::G4;
        if (it >= NI) break;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int sh = 16 * (p & 1), wd = p >> 1;
            const uint32_t c0 = (v[u][0][wd] >> sh) & 0xFFFFu, c1 = (v[u][1][wd] >> sh) & 0xFFFFu;
            const uint32_t c2 = (v[u][2][wd] >> sh) & 0xFFFFu, c3 = (v[u][3][wd] >> sh) & 0xFFFFu;
            xs[(r * S::X + 4 * xq + p + 1) * S::P + g] = make_uint2(c0 | (c1 << 16), c2 | (c3 << 16));
        }
    }
    for (int it = t; it < S::R * S::G4; it += 256)
        xs[(it / S::G4) * S::X * S::P + it % S::G4] = make_uint2(0u, 0u);
#pragma unroll
    for (int u = 0; u < UW; ++u) {
        const int it = t + 256 * u;
        if (it < NW) reinterpret_cast<uint4 *>(ws)[it] = wc[u];
    }
    __syncthreads();

    const int wv = t >> 6, l = t & 63, q = l >> 4, c = l & 15;
    f32x4 acc[G::MB][PW];
#pragma unroll
    for (int mb = 0; mb < G::MB; ++mb)
#pragma unroll
        for (int j = 0; j < PW; ++j) acc[mb][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < S::KB; ++kb) {
        const int k0 = 16 * kb + 4 * q;   // the lane's four reduction indices: k0 .. k0 + 3
        const int tap = k0 / S::CIP, g = (k0 - tap * S::CIP) >> 2;
        const int tc = tap < 9 ? tap : 0, ky = tc / 3, kx = tc - 3 * ky;
        bf16x4 av[G::MB];
#pragma unroll
        for (int mb = 0; mb < G::MB; ++mb)
            av[mb] = *reinterpret_cast<const bf16x4 *>(ws + (mb * 16 + c) * S::KROW + k0);
#pragma unroll
        for (int j = 0; j < PW; ++j) {
            const int blk = wv * PW + j, row = blk / BR, ox = (blk % BR) * 16 + c;
            bf16x4 bv = *reinterpret_cast<const bf16x4 *>(xs + ((2 * row + ky) * S::X + 2 * ox + kx) * S::P + g);
            if (tap >= 9) bv = bf16x4{0, 0, 0, 0};
#pragma unroll
            for (int mb = 0; mb < G::MB; ++mb) acc[mb][j] = mfma(av[mb], bv, acc[mb][j]);
        }
    }
#pragma unroll
    for (int j = 0; j < PW; ++j) {
        const int blk = wv * PW + j;
        const int p = (oy0 + blk / BR) * HO + (blk % BR) * 16 + c;
#pragma unroll
        for (int mb = 0; mb < G::MB; ++mb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int co = mb * 16 + 4 * q + i;
                out[((long long)b * CO + co) * G::HWO + p] = to_bf16(fmaxf(acc[mb][j][i] + bias[co], 0.0f));
            }
    }
}

// gap[b][c] = mean of a3[b][c]; z[b] = sum_c gap[b][c] wf[c] + bf, and,
// where asked for, the decision z[b] > 0 as flags[b] / decisions[b].  Eight
// lanes per channel, 32 positions each; the lane sums are combined by a
// butterfly, so the order is fixed and every lane of the eight holds the
// same total.
__global__ __launch_bounds__(256) void head_fwd(const uint16_t *__restrict__ a3, const float *__restrict__ theta,
                                               float *__restrict__ gap, float *__restrict__ logits,
                                               int *__restrict__ flags, uint8_t *__restrict__ decisions) {
    constexpr int HW = kH3 * kH3;
    static_assert(kC3 * 8 == 256 && HW == 8 * 32, "eight lanes of 32 positions per channel");
    typedef uint32_t u32x4a2 __attribute__((ext_vector_type(4), aligned(2)));
    __shared__ float part[kC3];
    const int b = blockIdx.x, t = threadIdx.x, ch = t >> 3;
    const uint16_t *p = a3 + ((long long)b * kC3 + ch) * HW + (t & 7) * 32;
    float s = 0.0f;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const u32x4a2 u = *reinterpret_cast<const u32x4a2 *>(p + 8 * v);
#pragma unroll
        for (int e = 0; e < 4; ++e) s += __uint_as_float(u[e] << 16) + __uint_as_float(u[e] & 0xFFFF0000u);
    }
    s += __shfl_xor(s, 1);
    s += __shfl_xor(s, 2);
    s += __shfl_xor(s, 4);
    const float g = s / (float)HW;
    if ((t & 7) == 0) {
        gap[b * kC3 + ch] = g;
        part[ch] = g * theta[kOffWf + ch];
    }
    __syncthreads();
    if (t < 64) {
        float z = t < kC3 ? part[t] : 0.0f;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) z += __shfl_xor(z, off);
        if (t == 0) {
            z += theta[kOffBf];
            logits[b] = z;
            if (flags) flags[b] = z > 0.0f;
            if (decisions) decisions[b] = (uint8_t)(z > 0.0f);
        }
    }
}

// ---------------------------------------------------------------- backward
// dz = (sigmoid(z) - y) / B, the per-sample loss, and the masked gradient
// of the last convolution: g3 = bf16(dz wf[c] / 256) where a3 > 0.
__global__ __launch_bounds__(256) void head_bwd(NetBuffers n) {
    constexpr int HW = kH3 * kH3;
    const int b = blockIdx.x;
    const float z = n.logits[b];
    const float y = n.labels[n.idx ? n.idx[b] : b];
    const float dz = (1.0f / (1.0f + expf(-z)) - y) / (float)n.B;
    if (threadIdx.x == 0) {
        n.dz[b] = dz;
        n.lossb[b] = fmaxf(z, 0.0f) - z * y + log1pf(expf(-fabsf(z)));
    }
    for (int i = threadIdx.x; i < kC3 * HW; i += blockDim.x) {
        const long long at = (long long)b * kC3 * HW + i;
        const float d = dz * n.theta[kOffWf + i / HW] / (float)HW;
        n.g3[at] = n.a3[at] != 0 ? to_bf16(d) : (uint16_t)0;
    }
}

// Head gradients and the mean loss: one wave, samples in order.
__global__ __launch_bounds__(64) void head_grad(NetBuffers n) {
    const int c = threadIdx.x;
    if (c < kC3) {
        float s = 0.0f;
        for (int b = 0; b < n.B; ++b) s += n.gap[b * kC3 + c] * n.dz[b];
        n.grad[kOffWf + c] = s;
    }
    if (c == 0) {
        float s = 0.0f, l = 0.0f;
        for (int b = 0; b < n.B; ++b) {
            s += n.dz[b];
            l += n.lossb[b];
        }
        n.grad[kOffBf] = s;
        if (n.loss) n.loss[0] = l / (float)n.B;
    }
}

// gin[b][ci][y][x] = bf16(sum_{co,ky,kx} w[co][ci][ky][kx] g[b][co][oy][ox]) where act[b][ci][y][x] > 0,
// over (oy, ox) with y = 2oy + ky - 1, x = 2ox + kx - 1.  GEMM rows = ci,
// columns = 16 input pixels, reduction over (co, ky, kx).
template <int CI, int CO, int HI>
__global__ __launch_bounds__(256) void conv_bwd_data(const uint16_t *__restrict__ g, const uint16_t *__restrict__ w,
                                                     const uint16_t *__restrict__ act, uint16_t *__restrict__ gin,
                                                     int B) {
    using G = Geo<CI, CO, HI>;
    constexpr int PB = G::HWI / 16, K = CO * 9, MB = CI / 16;
    static_assert(CI % 16 == 0, "input channels");
    const int wave = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + threadIdx.x / 64);
    if (wave >= B * PB) return;
    const int b = wave / PB, p0 = (wave % PB) * 16;
    const int l = threadIdx.x & 63, q = l >> 4, c = l & 15;
    const int p = p0 + c, y = p / HI, x = p % HI;
    const uint16_t *gb = g + (long long)b * CO * G::HWO;
    f32x4 acc[MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) acc[mb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
    for (int kb = 0; kb < K; kb += 16) {
        bf16x4 bv;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = kb + 4 * q + i;
            const int co = k / 9, t = k - 9 * co, ky = t / 3, kx = t - 3 * ky;
            const int ty = y + 1 - ky, tx = x + 1 - kx;
            const bool ok = ty >= 0 && tx >= 0 && !(ty & 1) && !(tx & 1) && ty < HI && tx < HI;
            bv[i] = ok ? (short)gb[co * G::HWO + (ty >> 1) * G::HO + (tx >> 1)] : (short)0;
        }
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            bf16x4 av;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int k = kb + 4 * q + i;
                const int co = k / 9, t = k - 9 * co;
                av[i] = (short)w[(co * CI + mb * 16 + c) * 9 + t];
            }
            acc[mb] = mfma(av, bv, acc[mb]);
        }
    }
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int ci = mb * 16 + 4 * q + i;
            const long long at = ((long long)b * CI + ci) * G::HWI + p;
            gin[at] = act[at] != 0 ? to_bf16(acc[mb][i]) : (uint16_t)0;
        }
}

// Weight and bias gradients, one split of the reduction per sample:
// partial[b][co][n] = sum over the output pixels of sample b of
// g[b][co][p] * X(p, n), X(p, n) = in[b][ci][2oy+ky-1][2ox+kx-1] for
// n = (ci, ky, kx) < CI*9 and X = 1 for n = CI*9 (the bias).
template <int CI, int CO, int HI>
__global__ __launch_bounds__(256) void conv_bwd_weight(const uint16_t *__restrict__ g, const uint16_t *__restrict__ in,
                                                       const int *__restrict__ idx, float *__restrict__ partial,
                                                       int B) {
    using G = Geo<CI, CO, HI>;
    const int wave = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + threadIdx.x / 64);
    if (wave >= B * G::NT) return;
    const int b = wave / G::NT, n0 = (wave % G::NT) * 16;
    const int l = threadIdx.x & 63, q = l >> 4, c = l & 15;
    const int n = n0 + c;
    const int ci = n / 9, t = n - 9 * ci, ky = t / 3, kx = t - 3 * ky;
    const uint16_t *ib = in + (long long)(idx ? idx[b] : b) * CI * G::HWI + (n < G::K ? ci * G::HWI : 0);
    const uint16_t *gb = g + (long long)b * CO * G::HWO;
    f32x4 acc[G::MB];
#pragma unroll
    for (int mb = 0; mb < G::MB; ++mb) acc[mb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
    for (int kb = 0; kb < G::HWO; kb += 16) {
        bf16x4 bv;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int p = kb + 4 * q + i, oy = p / G::HO, ox = p % G::HO;
            const int iy = 2 * oy + ky - 1, ix = 2 * ox + kx - 1;
            short v = 0;
            if (n < G::K) v = (iy >= 0 && ix >= 0) ? (short)ib[iy * HI + ix] : (short)0;
            else if (n == G::K) v = (short)0x3F80;   // 1.0
            bv[i] = v;
        }
#pragma unroll
        for (int mb = 0; mb < G::MB; ++mb) {
            // four consecutive pixels of channel mb*16 + c: one 8-byte load
            const bf16x4 av = *reinterpret_cast<const bf16x4 *>(gb + (mb * 16 + c) * G::HWO + kb + 4 * q);
            acc[mb] = mfma(av, bv, acc[mb]);
        }
    }
    if (n >= G::NW1) return;
#pragma unroll
    for (int mb = 0; mb < G::MB; ++mb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int co = mb * 16 + 4 * q + i;
            partial[((long long)b * CO + co) * G::NW1 + n] = acc[mb][i];
        }
}

// Sum the per-sample partials in sample order into the flat gradient.
template <int CI, int CO>
__global__ __launch_bounds__(256) void reduce_weight(const float *__restrict__ partial, float *__restrict__ grad,
                                                     int offw, int offb, int B) {
    constexpr int NW = CI * 9, NW1 = NW + 1;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= CO * NW1) return;
    float s = 0.0f;
    for (int b = 0; b < B; ++b) s += partial[(long long)b * CO * NW1 + i];
    const int co = i / NW1, n = i - co * NW1;
    if (n < NW) grad[offw + co * NW + n] = s;
    else grad[offb + co] = s;
}

// ---------------------------------------------------------------- AdamW
// Index in the bfloat16 copy of parameter i's second place, in the forward
// layout of its convolution's weights, or -1 for biases and the head.
template <int CI>
__device__ inline int forward_at_layer(int n, int perm) {
    const int co = n / (CI * 9), k = n - co * CI * 9, ci = k / 9, tap = k - 9 * ci;
    return perm + co * perm_row(CI) + tap * perm_cip(CI) + ci;
}
__device__ inline int forward_at(int i) {
    if (i >= kOffW1 && i < kOffB1) return forward_at_layer<kC0>(i - kOffW1, kPermW1);
    if (i >= kOffW2 && i < kOffB2) return forward_at_layer<kC1>(i - kOffW2, kPermW2);
    if (i >= kOffW3 && i < kOffB3) return forward_at_layer<kC2>(i - kOffW3, kPermW3);
    return -1;
}

// Decoupled weight decay on every parameter; refreshes the bfloat16 copy.
__global__ __launch_bounds__(256) void adamw(AdamArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const float g = a.grad[i];
    const float m = a.beta1 * a.m[i] + (1.0f - a.beta1) * g;
    const float v = a.beta2 * a.v[i] + (1.0f - a.beta2) * g * g;
    a.m[i] = m;
    a.v[i] = v;
    const float p = a.theta[i];
    const float np = p - a.lr * ((m / a.bc1) / (sqrtf(v / a.bc2) + a.eps) + a.wd * p);
    a.theta[i] = np;
    const uint16_t h = to_bf16(np);
    a.wbf[i] = h;
    const int j = forward_at(i);
    if (j >= 0) a.wbf[j] = h;
}

__global__ __launch_bounds__(256) void params_to_bf16(const float *theta, uint16_t *wbf) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kNParam) return;
    const uint16_t h = to_bf16(theta[i]);
    wbf[i] = h;
    const int j = forward_at(i);
    if (j >= 0) wbf[j] = h;
}

// ---------------------------------------------------------------- features
// Number of positions i in [0, n) with floor(i * cells / n) == c.
__device__ inline long long cell_span(long long c, long long n, long long cells) {
    return ((c + 1) * n + cells - 1) / cells - (c * n + cells - 1) / cells;
}

// Cell sums to bfloat16 features: (mean value) / maxval, (pixels with
// Z_1 != 0) / area, (Z_2 != 0) / area.  Feature set blockIdx.y covers
// image blockIdx.y / (gx gy) and, within it, region blockIdx.y % (gx gy)
// (row-major, gx regions per row) of kCells x kCells cells; the image's
// cell grid is gy kCells rows by gx kCells columns (gx = gy = 1: the whole
// image).  A workgroup takes kFinRows cell rows of one set; the cell
// spans of its rows and columns (64-bit divisions) are computed once into
// LDS.
constexpr int kFinRows = 16;
__global__ __launch_bounds__(256) void finish_features(Launch L, const unsigned long long *__restrict__ cells,
                                                       double maxval, uint16_t *__restrict__ feats, int gx,
                                                       int gy) {
    static_assert(kCells + kFinRows <= 256 && kCells % kFinRows == 0, "spans of one workgroup");
    __shared__ long long span_x[kCells], span_y[kFinRows];
    const int set = blockIdx.y, nreg = gx * gy;
    const int img = set / nreg, reg = set - img * nreg;
    const ImageJob &J = L.nimg == 1 ? L.one : L.jobs[img];
    const long long CX = (long long)gx * kCells, CY = (long long)gy * kCells;
    const int r0 = blockIdx.x * kFinRows;
    const long long cy0 = (long long)(reg / gx) * kCells + r0, cx0 = (long long)(reg % gx) * kCells;
    const int t = threadIdx.x;
    const unsigned long long *cs0 = cells + (long long)img * 2 * CX * CY + cy0 * CX + cx0;
    uint16_t *f = feats + (long long)set * kFeatC * kCellCount + r0 * kCells;
    // every cell's two sums are loaded before the spans and the first use
    constexpr int U = kFinRows * kCells / 256;
    static_assert(U * 256 == kFinRows * kCells, "whole cells per thread");
    unsigned long long sv[U], zz[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int j = t + 256 * u, r = j / kCells, x = j - r * kCells;
        sv[u] = cs0[r * CX + x];
        zz[u] = cs0[CX * CY + r * CX + x];
    }
    if (t < kCells) span_x[t] = cell_span(cx0 + t, J.img.W, CX);
    else if (t < kCells + kFinRows) span_y[t - kCells] = cell_span(cy0 + (t - kCells), J.img.H, CY);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int j = t + 256 * u, r = j / kCells, x = j - r * kCells;
        const long long area = span_y[r] * span_x[x];
        uint16_t f0 = 0, f1 = 0, f2 = 0;
        if (area > 0) {
            const double ar = (double)area;
            f0 = to_bf16((float)(((double)sv[u] / ar) / maxval));
            f1 = to_bf16((float)((double)(zz[u] & 0xFFFFFFFFull) / ar));
            f2 = to_bf16((float)((double)(zz[u] >> 32) / ar));
        }
        f[j] = f0;
        f[kCellCount + j] = f1;
        f[2 * kCellCount + j] = f2;
    }
}

// Clears n2 16-byte words (the cell sums: two per pair of cells).
__global__ __launch_bounds__(256) void zero_cells(ulonglong2 *p, long long n2) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n2) p[i] = make_ulonglong2(0ull, 0ull);
}

inline unsigned blocks(long long n, int t) { return (unsigned)((n + t - 1) / t); }

template <int CI, int CO, int HI, int TH>
hipError_t fwd(const uint16_t *in, const int *idx, const uint16_t *w, const float *bias, uint16_t *out, int B,
               hipStream_t s) {
    hipLaunchKernelGGL((conv_fwd<CI, CO, HI, TH>), dim3((unsigned)B * (HI / 2 / TH)), dim3(256), 0, s, in, idx, w,
                       bias, out, B);
    return hipGetLastError();
}

template <int CI, int CO, int HI>
hipError_t bwd_weight(const uint16_t *g, const uint16_t *in, const int *idx, float *partial, float *grad, int offw,
                      int offb, int B, hipStream_t s) {
    using G = Geo<CI, CO, HI>;
    hipLaunchKernelGGL((conv_bwd_weight<CI, CO, HI>), dim3(blocks((long long)B * G::NT, 4)), dim3(256), 0, s, g, in,
                       idx, partial, B);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((reduce_weight<CI, CO>), dim3(blocks(CO * G::NW1, 256)), dim3(256), 0, s, partial, grad, offw,
                       offb, B);
    return hipGetLastError();
}

template <int CI, int CO, int HI>
hipError_t bwd_data(const uint16_t *g, const uint16_t *w, const uint16_t *act, uint16_t *gin, int B, hipStream_t s) {
    using G = Geo<CI, CO, HI>;
    hipLaunchKernelGGL((conv_bwd_data<CI, CO, HI>), dim3(blocks((long long)B * (G::HWI / 16), 4)), dim3(256), 0, s, g,
                       w, act, gin, B);
    return hipGetLastError();
}

}  // namespace

long long partial_elems(int B) {
    const long long a = (long long)kC1 * Geo<kC0, kC1, kH0>::NW1;
    const long long b = (long long)kC2 * Geo<kC1, kC2, kH1>::NW1;
    const long long c = (long long)kC3 * Geo<kC2, kC3, kH2>::NW1;
    return (long long)B * (a > b ? (a > c ? a : c) : (b > c ? b : c));
}

hipError_t launch_zero_cells(unsigned long long *cells, long long nsets, hipStream_t s) {
    const long long n = nsets * 2 * kCellCount;
    static_assert(kCellCount % 2 == 0, "cell sums in 16-byte words");
    hipLaunchKernelGGL(zero_cells, dim3(blocks(n / 2, 256)), dim3(256), 0, s, reinterpret_cast<ulonglong2 *>(cells),
                       n / 2);
    return hipGetLastError();
}

hipError_t launch_finish_features(const Launch &L, const unsigned long long *cells, double maxval, uint16_t *feats,
                                  int gx, int gy, hipStream_t s) {
    hipLaunchKernelGGL(finish_features, dim3(kCells / kFinRows, L.nimg * gx * gy), dim3(256), 0, s, L, cells, maxval,
                       feats, gx, gy);
    return hipGetLastError();
}

hipError_t launch_forward(const NetBuffers &n, hipStream_t s, int *flags, uint8_t *decisions) {
    // conv_fwd copies each layer's weights in 16-byte chunks
    static_assert(kPermW1 % 8 == 0 && kPermW2 % 8 == 0 && kPermW3 % 8 == 0, "weight offsets");
    hipError_t e;
    // output rows per workgroup: 4, 4, 8 (measured against 8, 8 and 4, 16)
    if ((e = fwd<kC0, kC1, kH0, 4>(n.x0, n.idx, n.w + kPermW1, n.theta + kOffB1, n.a1, n.B, s)) != hipSuccess) return e;
    if ((e = fwd<kC1, kC2, kH1, 4>(n.a1, nullptr, n.w + kPermW2, n.theta + kOffB2, n.a2, n.B, s)) != hipSuccess) return e;
    if ((e = fwd<kC2, kC3, kH2, 8>(n.a2, nullptr, n.w + kPermW3, n.theta + kOffB3, n.a3, n.B, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(head_fwd, dim3(n.B), dim3(256), 0, s, n.a3, n.theta, n.gap, n.logits, flags, decisions);
    return hipGetLastError();
}

hipError_t launch_backward(const NetBuffers &n, hipStream_t s) {
    hipError_t e;
    hipLaunchKernelGGL(head_bwd, dim3(n.B), dim3(256), 0, s, n);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = bwd_weight<kC2, kC3, kH2>(n.g3, n.a2, nullptr, n.partial, n.grad, kOffW3, kOffB3, n.B, s)) != hipSuccess)
        return e;
    if ((e = bwd_data<kC2, kC3, kH2>(n.g3, n.w + kOffW3, n.a2, n.g2, n.B, s)) != hipSuccess) return e;
    if ((e = bwd_weight<kC1, kC2, kH1>(n.g2, n.a1, nullptr, n.partial, n.grad, kOffW2, kOffB2, n.B, s)) != hipSuccess)
        return e;
    if ((e = bwd_data<kC1, kC2, kH1>(n.g2, n.w + kOffW2, n.a1, n.g1, n.B, s)) != hipSuccess) return e;
    if ((e = bwd_weight<kC0, kC1, kH0>(n.g1, n.x0, n.idx, n.partial, n.grad, kOffW1, kOffB1, n.B, s)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(head_grad, dim3(1), dim3(64), 0, s, n);
    return hipGetLastError();
}

hipError_t launch_adamw(const AdamArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(adamw, dim3(blocks(a.n, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_params_to_bf16(const float *theta, uint16_t *wbf, hipStream_t s) {
    hipLaunchKernelGGL(params_to_bf16, dim3(blocks(kNParam, 256)), dim3(256), 0, s, theta, wbf);
    return hipGetLastError();
}

}  // namespace gate
}  // namespace logfx
