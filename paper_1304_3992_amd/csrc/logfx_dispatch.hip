// The finalize kernel and the run-time selection among the pass-kernel
// instantiation units (one per pair of mask radii, logfx_kernels_inst.hip).
#include "logfx_kernels.h"

#include <mutex>

#define LOGFX_RADII(X)                                                                            \
    X(1, 1) X(1, 2) X(2, 2) X(1, 3) X(2, 3) X(3, 3) X(1, 4) X(2, 4) X(3, 4) X(4, 4)

namespace logfx {

#define X(A, B)                                                                                   \
    hipError_t pass1_i_r##A##_##B(const Pass1Args<OrbitTapsI> &, int, int, hipStream_t, int *);  \
    hipError_t pass1_d_r##A##_##B(const Pass1Args<OrbitTapsD> &, int, int, hipStream_t, int *);  \
    hipError_t pass2_i_r##A##_##B(const Pass2Args<OrbitTapsI> &, int, hipStream_t, int *);        \
    hipError_t pass2_d_r##A##_##B(const Pass2Args<OrbitTapsD> &, int, hipStream_t, int *);
LOGFX_RADII(X)
#undef X

namespace kern {

// ------------------------------------------------------------- finalize
// One workgroup per image: fixed-order reduction of the image's tile sums.
// 1024 threads, so that the tiles of an 8192^2 image (about 4400) are read
// in one round of loads.
constexpr int kFinThreads = 1024;
__global__ __launch_bounds__(kFinThreads) void finalize_kernel(FinalizeArgs a) {
    __shared__ double sd[4][kFinThreads];
    __shared__ long long sc[2][kFinThreads];
    const int t = threadIdx.x;
    const int image = blockIdx.x;
    const ImageJob J = job_of(a.L, image);
    double s[4] = {0, 0, 0, 0};
    long long c[2] = {0, 0};
    // thread t adds tiles t, t + kFinThreads, ... in that order; U tiles'
    // loads are in flight at once (a tile past the end adds zeros, which
    // leaves the sums unchanged)
    constexpr int U = 8;
    for (int i0 = t; i0 < J.ntiles1; i0 += kFinThreads * U) {
        double v[U][4];
        long long w[U][2];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + kFinThreads * u;
            const long long at = (long long)J.base1 + i;
            const bool in = i < J.ntiles1;
#pragma unroll
            for (int k = 0; k < 4; ++k) v[u][k] = in ? a.partials[at * 4 + k] : 0.0;
            w[u][0] = in ? a.counts[at * 2] : 0;
            w[u][1] = in ? a.counts[at * 2 + 1] : 0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int k = 0; k < 4; ++k) s[k] += v[u][k];
            c[0] += w[u][0];
            c[1] += w[u][1];
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) sd[k][t] = s[k];
    sc[0][t] = c[0];
    sc[1][t] = c[1];
    __syncthreads();
    for (int off = kFinThreads / 2; off > 0; off >>= 1) {
        if (t < off) {
#pragma unroll
            for (int k = 0; k < 4; ++k) sd[k][t] += sd[k][t + off];
            sc[0][t] += sc[0][t + off];
            sc[1][t] += sc[1][t + off];
        }
        __syncthreads();
    }
    if (t == 0) {
        const long long npx = J.img.H * J.img.W;
        const double n = (double)npx;
        DevStats &st = a.stats[image];
        for (int j = 0; j < 2; ++j) {
            const double S = sd[j][0], Q = sd[2 + j][0];
            double var = npx > 1 ? (Q - S * (S / n)) / (n - 1.0) : 0.0;
            if (!(var > 0.0)) var = 0.0;
            const double sg = sqrt(var);
            const double T = a.std_mode == 0 ? a.std_k * sg : a.abs_thr[j];
            st.sum[j] = S;
            st.sumsq[j] = Q;
            st.sigma[j] = sg;
            st.thresh[j] = T;
            st.thr72[j] = 72.0 * T * T;
            st.zc[j] = sc[j][0];
        }
    }
}

}  // namespace kern

hipError_t launch_pass1_i(int ra, int rb, const Pass1Args<OrbitTapsI> &a, int mode, int grid,
                          hipStream_t s, int *max_grid) {
#define X(A, B) if (ra == A && rb == B) return pass1_i_r##A##_##B(a, mode, grid, s, max_grid);
    LOGFX_RADII(X)
#undef X
    return hipErrorInvalidValue;
}
hipError_t launch_pass1_d(int ra, int rb, const Pass1Args<OrbitTapsD> &a, int mode, int grid,
                          hipStream_t s, int *max_grid) {
#define X(A, B) if (ra == A && rb == B) return pass1_d_r##A##_##B(a, mode, grid, s, max_grid);
    LOGFX_RADII(X)
#undef X
    return hipErrorInvalidValue;
}
hipError_t launch_pass2_i(int ra, int rb, const Pass2Args<OrbitTapsI> &a, int grid, hipStream_t s,
                          int *max_grid) {
#define X(A, B) if (ra == A && rb == B) return pass2_i_r##A##_##B(a, grid, s, max_grid);
    LOGFX_RADII(X)
#undef X
    return hipErrorInvalidValue;
}
hipError_t launch_pass2_d(int ra, int rb, const Pass2Args<OrbitTapsD> &a, int grid, hipStream_t s,
                          int *max_grid) {
#define X(A, B) if (ra == A && rb == B) return pass2_d_r##A##_##B(a, grid, s, max_grid);
    LOGFX_RADII(X)
#undef X
    return hipErrorInvalidValue;
}
// The scratch of logfx_extract_noalloc: every call on a device shares its
// copy, which keeps the last call's contents (each pass writes every slot it
// later reads, so nothing needs clearing).
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

hipError_t noalloc_scratch(int device, void **ptr) {
    static std::mutex mu;
    static void *addr[64] = {};
    if (device < 0 || device >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = p;
    }
    *ptr = addr[device];
    return hipSuccess;
}

hipError_t launch_finalize(const FinalizeArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(kern::finalize_kernel, dim3(a.L.nimg), dim3(kern::kFinThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace logfx
