// Pass 2 on stored crossing strengths: E_j = [3x3 deviation of Z_j > T_j]
// (eq. (2), Sec. 4.1), E = E_1 OR E_2, F = hybrid median of E (Sec. 3.4).
//
// Pass 1 has written the pair (Z_1, Z_2) of every pixel to HBM (8 bytes per
// pixel on the integer path), so this pass computes no LoG: each lane of a
// wave reads its column's pairs, six rows ahead, with clamp-to-edge
// coordinates (the columns and rows outside the image read the edge
// pixel's pair, which is the clamped operand of the deviation), keeps a
// ring of three rows of the deviation's row sums (the neighbours from the
// adjacent lanes), and continues exactly as the pass that
// recomputes the strengths: same FP64 operations in the same order, so the
// two passes give the same output bit for bit.  No LDS; halo 3 columns
// (median 2 + deviation 1), 58 output columns per wave.
#include "logfx_kernels.h"

namespace logfx {
namespace kern {

template <class Acc, int MED, bool LOOP>
__global__ __launch_bounds__(256) void pass2z_kernel(Pass2Args<typename AccOps<Acc>::Taps> a) {
    using ZT = typename ZStore<Acc>::T;
    __shared__ int redc[2][8];
    constexpr int HL = kHalo2Z, OW = kWave - 2 * HL, TW = tile_out_width(HL);
    constexpr int G = 6;   // rows read ahead of their use (a multiple of the 3-row ring)

    auto tile = [&](const int item, auto medc) __attribute__((always_inline)) {
        constexpr int M = decltype(medc)::value;
        const int image = a.L.nimg == 1 ? 0 : a.L.owner2[item];
        const ImageJob J = job_of(a.L, image);
        const int H = (int)J.img.H, W = (int)J.img.W;
        const int tile = item - J.base2, tx = tile % J.tiles_x2, ty = tile / J.tiles_x2;
        const int x0 = tx * TW, y0 = ty * a.rows, Rv = min(a.rows, H - y0);
        const int lane = threadIdx.x & (kWave - 1);
        const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
        const int base = x0 + wave * OW - HL, xc = base + lane;
        const bool outc = lane >= HL && lane < HL + OW && xc < W;
        const ZT *zcol = static_cast<const ZT *>(a.zmap) + J.zoff + min(max(xc, 0), W - 1);

        const double thr72_0 = a.stats[image].thr72[0], thr72_1 = a.stats[image].thr72[1];
        const int lo_lane = base < 0 ? -base : 0;
        const int hi_lane = min(max(W - 1 - base, 0), kWave - 1);
        const uint64_t mybit = 1ull << lane;
        const uint64_t outmask = __ballot(outc);

        double Zs[2][3] = {{0, 0, 0}, {0, 0, 0}};  // deviation row sums, rows t-3, t-2, t-1
        double Zq[2][3] = {{0, 0, 0}, {0, 0, 0}};
        uint64_t e[5] = {0, 0, 0, 0, 0};           // rows t-6 .. t-2
        int ecnt = 0, fcnt = 0;
        // step si reads Z row t - 1 = y0 - 3 + si; rows y0-3 .. y0+Rv+2
        const int nsteps = Rv + 2 * HL;
        const int t0 = y0 - 2;
        uint8_t *orow = J.out + (long long)(t0 - 4) * J.out_pitch + xc;
        long long opitch;
        asm("v_mov_b64 %0, %1" : "=v"(opitch) : "s"(J.out_pitch));

        auto step = [&](const int si, const ZT &zv, auto clamp) __attribute__((always_inline)) {
            constexpr bool C = decltype(clamp)::value;
            const int t = t0 + si;
            double zn[2];
            ZStore<Acc>::get(zv, zn[0], zn[1]);
#pragma unroll
            for (int j = 0; j < 2; ++j) {   // row sums of row t - 1 (columns clamped by the loads)
                double hs, hq;
                dev_row(from_left(zn[j]), zn[j], from_right(zn[j]), hs, hq);
                Zs[j][0] = Zs[j][1];
                Zs[j][1] = Zs[j][2];
                Zs[j][2] = hs;
                Zq[j][0] = Zq[j][1];
                Zq[j][1] = Zq[j][2];
                Zq[j][2] = hq;
            }
            bool ej = false;
#pragma unroll
            for (int j = 0; j < 2; ++j)     // extraction of row t - 2: 3x3 deviation of Z
                ej = ej || (dev_72var(Zs[j], Zq[j]) > (j == 0 ? thr72_0 : thr72_1));
            ring_push<C>(e, clamp_bits(__ballot(ej), lo_lane, hi_lane), t - 2, H);
            uint64_t f;   // output row t - 4 (from the seventh step on)
            if constexpr (M == 0) f = e[2];
            else f = hybrid_median<M>(e);
            if (si >= 6) {
                if (outc) *orow = (uint8_t)((f & mybit) != 0);
                fcnt += __popcll(f & outmask);
                ecnt += __popcll(e[2] & outmask);
            }
            orow += opitch;
        };
        auto run = [&](auto clamp) __attribute__((always_inline)) {
            // full groups unrolled (loads first, the ring rotates by
            // renaming), the rest one step at a time; no step runs under a
            // condition, which keeps the median's bit rows in scalar registers
            int si0 = 0;
            for (; si0 + G <= nsteps; si0 += G) {
                ZT q[G];
#pragma unroll
                for (int k = 0; k < G; ++k) {
                    const int row = min(max(t0 - 1 + si0 + k, 0), H - 1);
                    q[k] = zcol[(long long)row * W];
                }
#pragma unroll
                for (int k = 0; k < G; ++k) step(si0 + k, q[k], clamp);
            }
            for (; si0 < nsteps; ++si0) {
                const int row = min(max(t0 - 1 + si0, 0), H - 1);
                step(si0, zcol[(long long)row * W], clamp);
            }
        };
        // the E rows y0-2 .. y0+Rv+1 the output uses lie inside the image:
        // no row clamping of the extracted bits
        if (y0 - 2 >= 0 && y0 + Rv + 1 <= H - 1) run(bool_c<false>{});
        else run(bool_c<true>{});

        const int w = threadIdx.x / kWave;
        if (lane == 0) {
            redc[0][w] = ecnt;
            redc[1][w] = fcnt;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int s0 = 0, s1 = 0;
            for (int k = 0; k < (int)(blockDim.x / kWave); ++k) {
                s0 += redc[0][k];
                s1 += redc[1][k];
            }
            a.counts[(long long)item * 2] = s0;
            a.counts[(long long)item * 2 + 1] = s1;
        }
        __syncthreads();   // the reduction buffer is reused by the next tile
    };
    for_each_tile<LOOP>(a.L.total2, [&](const int item) __attribute__((always_inline)) {
        if constexpr (MED >= 0) {
            tile(item, int_c<MED>{});
        } else {   // gated: the median of each image as its flag says
            const int image = a.L.nimg == 1 ? 0 : a.L.owner2[item];
            if (a.med_flags[image]) tile(item, int_c<-MED>{});
            else tile(item, int_c<0>{});
        }
    });
}

template <class Acc, int MED>
hipError_t p2z(const Pass2Args<typename AccOps<Acc>::Taps> &a, int grid, hipStream_t s, int *max_grid) {
    constexpr bool CAN_LOOP = MED >= 0;   // gated variants run one tile per workgroup
    if (max_grid) return occupancy(pass2z_kernel<Acc, MED, CAN_LOOP>, 0, max_grid);
    if (!CAN_LOOP || grid >= a.L.total2)
        hipLaunchKernelGGL((pass2z_kernel<Acc, MED, false>), dim3(a.L.total2), dim3(kTileWaves * kWave), 0, s, a);
    else
        hipLaunchKernelGGL((pass2z_kernel<Acc, MED, CAN_LOOP>), dim3(grid), dim3(kTileWaves * kWave), 0, s, a);
    return hipGetLastError();
}

template <class Acc>
hipError_t p2z_any(const Pass2Args<typename AccOps<Acc>::Taps> &a, int grid, hipStream_t s, int *max_grid) {
    if (a.med_flags) return a.median_size == 3 ? p2z<Acc, -3>(a, grid, s, max_grid) : p2z<Acc, -5>(a, grid, s, max_grid);
    if (!a.smooth) return p2z<Acc, 0>(a, grid, s, max_grid);
    return a.median_size == 3 ? p2z<Acc, 3>(a, grid, s, max_grid) : p2z<Acc, 5>(a, grid, s, max_grid);
}

}  // namespace kern

hipError_t launch_pass2z_i(const Pass2Args<OrbitTapsI> &a, int grid, hipStream_t s, int *max_grid) {
    return kern::p2z_any<int>(a, grid, s, max_grid);
}
hipError_t launch_pass2z_d(const Pass2Args<OrbitTapsD> &a, int grid, hipStream_t s, int *max_grid) {
    return kern::p2z_any<double>(a, grid, s, max_grid);
}

}  // namespace logfx
