// The smoothing gate: a small CNN that decides per image whether the hybrid
// median is applied.  The paper leaves that choice to the user, according
// to the noise in the extracted map (abstract; Sec. 4).
//
// Network: three 3x3 convolutions of stride 2 with zero padding
// (3 -> 16 -> 32 -> 32 channels, 128 -> 64 -> 32 -> 16), ReLU after each,
// global average pooling and a linear layer to one logit.  The convolutions
// run as implicit GEMMs on v_mfma_f32_16x16x16_bf16: bfloat16 operands
// gathered straight from the activation maps, FP32 accumulation, one wave
// per 16 x (all output channels) block.  Stored activations and their
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
// image, reduction over (ci, ky, kx).  A wave takes PW consecutive blocks of
// 16 pixels of one image: each weight fragment is loaded once for the PW
// products that use it.
template <int CI, int CO, int HI, int PW>
__global__ __launch_bounds__(256) void conv_fwd(const uint16_t *__restrict__ in, const int *__restrict__ idx,
                                                const uint16_t *__restrict__ w, const float *__restrict__ bias,
                                                uint16_t *__restrict__ out, int B) {
    using G = Geo<CI, CO, HI>;
    constexpr int PB = G::HWO / 16;   // 16-pixel blocks per image
    static_assert(PB % PW == 0, "whole blocks per wave");
    const int wave = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + threadIdx.x / 64);
    if (wave >= B * (PB / PW)) return;
    const int b = wave / (PB / PW), pb0 = (wave % (PB / PW)) * PW;
    const int l = threadIdx.x & 63, q = l >> 4, c = l & 15;
    const uint16_t *ib = in + (long long)(idx ? idx[b] : b) * CI * G::HWI;
    f32x4 acc[G::MB][PW];
#pragma unroll
    for (int mb = 0; mb < G::MB; ++mb)
#pragma unroll
        for (int j = 0; j < PW; ++j) acc[mb][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < G::KP; kb += 16) {
        bf16x4 av[G::MB];
#pragma unroll
        for (int mb = 0; mb < G::MB; ++mb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int k = kb + 4 * q + i;
                av[mb][i] = k < G::K ? (short)w[(mb * 16 + c) * G::K + k] : (short)0;
            }
#pragma unroll
        for (int j = 0; j < PW; ++j) {
            const int p = (pb0 + j) * 16 + c, oy = p / G::HO, ox = p % G::HO;
            bf16x4 bv;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int k = kb + 4 * q + i;
                const int ci = k / 9, t = k - 9 * ci, ky = t / 3, kx = t - 3 * ky;
                const int iy = 2 * oy + ky - 1, ix = 2 * ox + kx - 1;   // < HI always
                bv[i] = (k < G::K && iy >= 0 && ix >= 0) ? (short)ib[ci * G::HWI + iy * HI + ix] : (short)0;
            }
#pragma unroll
            for (int mb = 0; mb < G::MB; ++mb) acc[mb][j] = mfma(av[mb], bv, acc[mb][j]);
        }
    }
#pragma unroll
    for (int j = 0; j < PW; ++j) {
        const int p = (pb0 + j) * 16 + c;
#pragma unroll
        for (int mb = 0; mb < G::MB; ++mb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int co = mb * 16 + 4 * q + i;
                out[((long long)b * CO + co) * G::HWO + p] = to_bf16(fmaxf(acc[mb][j][i] + bias[co], 0.0f));
            }
    }
}

// gap[b][c] = mean of a3[b][c]; z[b] = sum_c gap[b][c] wf[c] + bf
__global__ __launch_bounds__(64) void head_fwd(const uint16_t *__restrict__ a3, const float *__restrict__ theta,
                                              float *__restrict__ gap, float *__restrict__ logits) {
    constexpr int HW = kH3 * kH3;
    const int b = blockIdx.x, c = threadIdx.x;
    float g = 0.0f;
    if (c < kC3) {
        const uint16_t *p = a3 + ((long long)b * kC3 + c) * HW;
        float s = 0.0f;
        for (int i = 0; i < HW; ++i) s += from_bf16(p[i]);
        g = s / (float)HW;
        gap[b * kC3 + c] = g;
    }
    float t = c < kC3 ? g * theta[kOffWf + c] : 0.0f;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off);
    if (c == 0) logits[b] = t + theta[kOffBf];
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
    a.wbf[i] = to_bf16(np);
}

__global__ __launch_bounds__(256) void to_bf16_kernel(const float *src, uint16_t *dst, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = to_bf16(src[i]);
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
// image).
__global__ __launch_bounds__(256) void finish_features(Launch L, const unsigned long long *__restrict__ cells,
                                                       double maxval, uint16_t *__restrict__ feats, int gx,
                                                       int gy) {
    const int set = blockIdx.y, nreg = gx * gy;
    const int img = set / nreg, reg = set - img * nreg;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kCellCount) return;
    const ImageJob &J = L.nimg == 1 ? L.one : L.jobs[img];
    const long long CX = (long long)gx * kCells, CY = (long long)gy * kCells;
    const long long cy = (long long)(reg / gx) * kCells + i / kCells;
    const long long cx = (long long)(reg % gx) * kCells + i % kCells;
    const long long area = cell_span(cy, J.img.H, CY) * cell_span(cx, J.img.W, CX);
    const unsigned long long *cs = cells + (long long)img * 2 * CX * CY + cy * CX + cx;
    uint16_t *f = feats + (long long)set * kFeatC * kCellCount;
    if (area <= 0) {
        f[i] = f[kCellCount + i] = f[2 * kCellCount + i] = 0;
        return;
    }
    const double ar = (double)area;
    const unsigned long long zz = cs[CX * CY];
    f[i] = to_bf16((float)(((double)cs[0] / ar) / maxval));
    f[kCellCount + i] = to_bf16((float)((double)(zz & 0xFFFFFFFFull) / ar));
    f[2 * kCellCount + i] = to_bf16((float)((double)(zz >> 32) / ar));
}

__global__ __launch_bounds__(256) void zero_u64(unsigned long long *p, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ __launch_bounds__(256) void decide(const float *logits, int *flags, uint8_t *decisions, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int d = logits[i] > 0.0f;
    if (flags) flags[i] = d;
    if (decisions) decisions[i] = (uint8_t)d;
}

inline unsigned blocks(long long n, int t) { return (unsigned)((n + t - 1) / t); }

template <int CI, int CO, int HI, int PW>
hipError_t fwd(const uint16_t *in, const int *idx, const uint16_t *w, const float *bias, uint16_t *out, int B,
               hipStream_t s) {
    using G = Geo<CI, CO, HI>;
    hipLaunchKernelGGL((conv_fwd<CI, CO, HI, PW>), dim3(blocks((long long)B * (G::HWO / 16 / PW), 4)), dim3(256), 0, s,
                       in, idx, w, bias, out, B);
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
    hipLaunchKernelGGL(zero_u64, dim3(blocks(n, 256)), dim3(256), 0, s, cells, n);
    return hipGetLastError();
}

hipError_t launch_finish_features(const Launch &L, const unsigned long long *cells, double maxval, uint16_t *feats,
                                  int gx, int gy, hipStream_t s) {
    hipLaunchKernelGGL(finish_features, dim3(blocks(kCellCount, 256), L.nimg * gx * gy), dim3(256), 0, s, L, cells,
                       maxval, feats, gx, gy);
    return hipGetLastError();
}

hipError_t launch_forward(const NetBuffers &n, hipStream_t s) {
    hipError_t e;
    if ((e = fwd<kC0, kC1, kH0, 4>(n.x0, n.idx, n.w + kOffW1, n.theta + kOffB1, n.a1, n.B, s)) != hipSuccess) return e;
    if ((e = fwd<kC1, kC2, kH1, 4>(n.a1, nullptr, n.w + kOffW2, n.theta + kOffB2, n.a2, n.B, s)) != hipSuccess) return e;
    if ((e = fwd<kC2, kC3, kH2, 2>(n.a2, nullptr, n.w + kOffW3, n.theta + kOffB3, n.a3, n.B, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(head_fwd, dim3(n.B), dim3(64), 0, s, n.a3, n.theta, n.gap, n.logits);
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

hipError_t launch_to_bf16(const float *src, uint16_t *dst, int n, hipStream_t s) {
    hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks(n, 256)), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_decide(const float *logits, int *flags, uint8_t *decisions, int n, hipStream_t s) {
    hipLaunchKernelGGL(decide, dim3(blocks(n, 256)), dim3(256), 0, s, logits, flags, decisions, n);
    return hipGetLastError();
}

}  // namespace gate
}  // namespace logfx
