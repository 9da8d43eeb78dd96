// Internal declarations of the smoothing gate: per-image features from
// pass 1, a three-layer strided CNN on MFMA, its backward pass and AdamW.
// Not part of the public ABI (include/logfx.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "logfx_internal.h"

namespace logfx {
namespace gate {

constexpr int kCells = 128;                  // feature grid: kCells x kCells cells per image
constexpr int kCellCount = kCells * kCells;
constexpr int kFeatC = 3;                    // mean value, crossing density of mask 1, of mask 2

// Layer shapes: 3x3 convolutions, stride 2, zero padding 1, ReLU.
//   conv1 3 -> 16 channels, 128 -> 64;  conv2 16 -> 32, 64 -> 32;  conv3 32 -> 32, 32 -> 16
// then the mean over the 16 x 16 positions and a linear map 32 -> 1.
constexpr int kC0 = kFeatC, kC1 = 16, kC2 = 32, kC3 = 32;
constexpr int kH0 = kCells, kH1 = kH0 / 2, kH2 = kH1 / 2, kH3 = kH2 / 2;

// Flat parameter vector (FP32 master copy), in this order:
//   w1[16][3][3][3] b1[16] w2[32][16][3][3] b2[32] w3[32][32][3][3] b3[32] wf[32] bf[1]
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kC1 * kC0 * 9;
constexpr int kOffW2 = kOffB1 + kC1;
constexpr int kOffB2 = kOffW2 + kC2 * kC1 * 9;
constexpr int kOffW3 = kOffB2 + kC2;
constexpr int kOffB3 = kOffW3 + kC3 * kC2 * 9;
constexpr int kOffWf = kOffB3 + kC3;
constexpr int kOffBf = kOffWf + kC3;
constexpr int kNParam = kOffBf + 1;          // 14369

// The bfloat16 copy of the parameters holds the flat vector and after it,
// for the forward kernels, each convolution's weights again as
// [co][tap * cip + ci] rows of perm_row(CI) entries: cip = CI rounded up to
// a multiple of 4, the row rounded up to whole 16-deep reduction blocks
// plus 8 (so that rows start 2 (mod 4) 8-byte words apart); the padding
// entries are zero.
constexpr int perm_cip(int ci) { return (ci + 3) / 4 * 4; }
constexpr int perm_row(int ci) { return (9 * perm_cip(ci) + 15) / 16 * 16 + 8; }
constexpr int kPermW1 = (kNParam + 7) / 8 * 8;
constexpr int kPermW2 = kPermW1 + kC1 * perm_row(kC0);
constexpr int kPermW3 = kPermW2 + kC2 * perm_row(kC1);
constexpr int kWbfElems = kPermW3 + kC3 * perm_row(kC2);

// Per-cell sums that pass 1 accumulates for every image (feature mode):
// [image][2][kCellCount] (or [2][gy kCells][gx kCells] for one image whose
// gx x gy regions the gate decides one by one) of
//   plane 0: sum of pixel values,
//   plane 1: (pixels with Z_1 != 0) + 2^32 * (pixels with Z_2 != 0).
// Plane 1 needs every cell to hold fewer than 2^32 pixels (checked on the host).
struct CellSink {
    unsigned long long *cells;   // nullptr: no feature accumulation
};

// Activations and gradients of one batch, bfloat16 bits, [B][C][H][H].
struct NetBuffers {
    const uint16_t *x0;      // features [N][3][128][128] (indexed through idx)
    const int *idx;          // [B] sample of each batch row, or nullptr (row b = sample b)
    const uint16_t *w;       // bfloat16 copy of the parameters (kWbfElems entries)
    const float *theta;      // FP32 parameters (biases, head)
    uint16_t *a1, *a2, *a3;  // ReLU outputs
    uint16_t *g1, *g2, *g3;  // masked gradients w.r.t. the pre-activations
    float *gap;              // [B][32]
    float *logits;           // [B]
    float *dz;               // [B] d loss / d logit
    float *lossb;            // [B] per-sample loss
    const float *labels;     // [N] (indexed through idx)
    float *grad;             // [kNParam]
    float *loss;             // [1] mean loss, or nullptr
    float *partial;          // split-K partial weight gradients
    int B;
};

// Workspace elements of NetBuffers for a batch of B rows.
constexpr long long act_elems(int B) {
    return (long long)B * (kC1 * kH1 * kH1 + kC2 * kH2 * kH2 + kC3 * kH3 * kH3);
}
long long partial_elems(int B);

struct AdamArgs {
    float *theta, *m, *v;
    const float *grad;
    uint16_t *wbf;        // refreshed bfloat16 copy (kWbfElems: flat, then the forward layout)
    float lr, beta1, beta2, eps, wd, bc1, bc2;   // bc = 1 - beta^t
    int n;
};

// Launchers (logfx_gate.hip).  They return hipSuccess or the launch error.
hipError_t launch_zero_cells(unsigned long long *cells, long long nsets, hipStream_t s);
// Features of the images of a launch: bf16 [nimg][gy gx][3][128][128] from
// the cell sums (gx x gy regions per image, 1 x 1 for whole images).
hipError_t launch_finish_features(const Launch &L, const unsigned long long *cells, double maxval,
                                  uint16_t *feats, int gx, int gy, hipStream_t s);
// The logits of the batch and, for non-null flags / decisions, the
// decisions flags[b] = decisions[b] = logits[b] > 0.
hipError_t launch_forward(const NetBuffers &n, hipStream_t s, int *flags = nullptr, uint8_t *decisions = nullptr);
hipError_t launch_backward(const NetBuffers &n, hipStream_t s);   // after launch_forward
hipError_t launch_adamw(const AdamArgs &a, hipStream_t s);
// wbf (kWbfElems, its padding already zero) from the FP32 parameters.
hipError_t launch_params_to_bf16(const float *theta, uint16_t *wbf, hipStream_t s);

}  // namespace gate
}  // namespace logfx
