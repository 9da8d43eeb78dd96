// Pass 2 on stored crossing strengths: E_j = [3x3 deviation of Z_j > T_j]
// (eq. (2), Sec. 4.1), E = E_1 OR E_2, F = hybrid median of E (Sec. 3.4).
//
// Pass 1 has written the pair (Z_1, Z_2) of every pixel to HBM (8 bytes per
// pixel on the integer path), so this pass computes no LoG: each lane of a
// wave reads its column's pairs, six rows ahead, with clamp-to-edge
// coordinates (the columns and rows outside the image read the edge
// pixel's pair, which is the clamped operand of the deviation), keeps a
// ring of three rows of the deviation's row sums (the neighbours from the
// adjacent lanes), and runs the same FP64 operations in the same order as
// the pass that recomputes the strengths, so the two passes give the same
// output bit for bit.  No LDS; halo 3 columns (median 2 + deviation 1), 58
// output columns per wave.
//
// Each lane collects the E bits of its own column in 32-bit words (bit k =
// row k of the word).  Once 36 rows past a word's start are known, the
// hybrid median of the word's 32 output rows is taken on whole words: a
// row offset is a funnel shift of two consecutive words, a column offset a
// lane shift, and each logic operation treats 32 pixels.
//
// With the 5x5 first stage (Sec. 4.1, std5_max >= 0) a pixel is extracted
// only if its 5x5 deviation also exceeds std5_max: a ring of five rows of
// 5-wide row sums beside the 3-wide ones, halo 4 (56 output columns).
#include "logfx_kernels.h"

namespace logfx {
namespace kern {

typedef __attribute__((address_space(1))) uint8_t GlobalU8;
// Bits s .. s + 31 of the 64-bit word hi:lo.
__device__ inline unsigned funnel(unsigned hi, unsigned lo, int s) { return __builtin_amdgcn_alignbit(hi, lo, s); }

// Hybrid median (window M = 3 or 5) of the 32 pixels of a column word:
// bit k of w1:w0 >> 2 is the centre of output row k, bits k .. k + 4 its
// column window; the other columns come from the neighbouring lanes.
template <int M>
__device__ inline unsigned median_word(unsigned w0, unsigned w1) {
    const unsigned c = funnel(w1, w0, 2);
    const unsigned l0 = from_left(w0), l1 = from_left(w1);     // column x - 1
    const unsigned r0 = from_right(w0), r1 = from_right(w1);   // column x + 1
    if constexpr (M == 3) {
        const unsigned p[4] = {funnel(l1, l0, 2), funnel(r1, r0, 2), funnel(w1, w0, 1), funnel(w1, w0, 3)};
        const unsigned x[4] = {funnel(l1, l0, 1), funnel(r1, r0, 1), funnel(l1, l0, 3), funnel(r1, r0, 3)};
        return hybrid_median_bits<3>(c, p, x);
    } else {
        const unsigned ll0 = from_left(l0), ll1 = from_left(l1);     // column x - 2
        const unsigned rr0 = from_right(r0), rr1 = from_right(r1);   // column x + 2
        const unsigned p[8] = {funnel(ll1, ll0, 2), funnel(l1, l0, 2), funnel(r1, r0, 2), funnel(rr1, rr0, 2),
                               w0, funnel(w1, w0, 1), funnel(w1, w0, 3), funnel(w1, w0, 4)};
        const unsigned x[8] = {ll0, rr0, funnel(l1, l0, 1), funnel(r1, r0, 1),
                               funnel(l1, l0, 3), funnel(r1, r0, 3), funnel(ll1, ll0, 4), funnel(rr1, rr0, 4)};
        return hybrid_median_bits<5>(c, p, x);
    }
}

// Row sums of the 5x5 deviation (the 5x5 first stage, Sec. 4.1): the 3x3
// row sums (s, q) of the pixel plus its neighbours two columns away.
__device__ inline void dev_row5(double zl2, double zr2, double s, double q, double &s5, double &q5) {
    s5 = s + (zl2 + zr2);
    q5 = __fma_rn(zr2, zr2, __fma_rn(zl2, zl2, q));
}
// 600 s5^2 = 25 sum z^2 - (sum z)^2 over the five rows of the window.
__device__ inline double dev_600var(const double (&s)[5], const double (&q)[5]) {
    const double S = (((s[0] + s[1]) + s[2]) + s[3]) + s[4];
    const double Q = (((q[0] + q[1]) + q[2]) + q[3]) + q[4];
    return __fma_rn(-S, S, 25.0 * Q);
}

// S5: with the 5x5 first stage, E_j(p) also needs the 5x5 deviation of Z_j
// above std5_max; the halo grows to 4 columns (56 output columns per wave).
template <class Acc, int MED, bool LOOP, bool S5>
__global__ __launch_bounds__(256) void pass2z_kernel(Pass2Args<typename AccOps<Acc>::Taps> a) {
    using ZT = typename ZStore<Acc>::T;
    __shared__ int redc[2][8];
    constexpr int HL = S5 ? kHalo2Z5 : kHalo2Z, OW = kWave - 2 * HL, TW = tile_out_width(HL);
    constexpr int WR = S5 ? 2 : 1;        // half-height of the widest deviation window
    constexpr int NR = 2 * WR + 1;        // rows of row sums kept
    constexpr int G = S5 ? 5 : 6;         // rows read ahead of their use (a multiple of the ring)

    // mixed: (gated per region) the tile's output pixels span regions, so
    // each pixel takes F or E by its own region's flag
    auto tile = [&](const int item, auto medc, const bool mixed) __attribute__((always_inline)) {
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
        const unsigned outm = outc ? ~0u : 0u;
        // the output map: the caller's, or the scratch map of a median cascade
        uint8_t *const obase = a.out_map ? a.out_map + J.zoff : J.out;
        const long long opitch = a.out_map ? (long long)W : J.out_pitch;

        // gated per region: the region column of the lane's (clamped) column
        int rx = 0;
        if constexpr (MED < 0) {
            if (mixed) rx = min(max(xc, 0), W - 1) / a.region;
        }
        const double thr600_0 = a.thr600[0], thr600_1 = a.thr600[1];
        double Zs[2][NR] = {}, Zq[2][NR] = {};   // 3x3 deviation row sums of the last NR rows read
        double Ws[2][NR] = {}, Wq[2][NR] = {};   // 5x5 deviation row sums (S5)
        // E bits of the lane's column: bit k of elo (of ehi) is E row
        // y0 - 2 + wb + k (+ 32); wb is the first output row, relative to
        // y0, of the next word to emit
        unsigned elo = 0, ehi = 0;
        int wb = 0;
        bool last = false;                // E bit of the previous row
        unsigned ecnt = 0, fcnt = 0;      // per lane, output pixels only
        // step si reads Z row y0 - HL + si and extracts E row y0 - HL - WR + si
        const int nsteps = Rv + 2 * HL;

        // F of output rows y0 + wb .. y0 + wb + n - 1 (n <= 32, E rows up to
        // y0 + wb + n + 1 present)
        auto emit = [&](const int n) __attribute__((always_inline)) {
            unsigned w0 = elo, w1 = ehi;
            if (lo_lane > 0) {   // columns left of the image repeat column 0
                const unsigned s0 = __builtin_amdgcn_readlane(w0, lo_lane);
                const unsigned s1 = __builtin_amdgcn_readlane(w1, lo_lane);
                w0 = lane < lo_lane ? s0 : w0;
                w1 = lane < lo_lane ? s1 : w1;
            }
            if (hi_lane < kWave - 1) {   // columns right of the image repeat column W - 1
                const unsigned s0 = __builtin_amdgcn_readlane(w0, hi_lane);
                const unsigned s1 = __builtin_amdgcn_readlane(w1, hi_lane);
                w0 = lane > hi_lane ? s0 : w0;
                w1 = lane > hi_lane ? s1 : w1;
            }
            // bit k of funnel(.., 2 + d): E row y0 + wb + k + d
            const unsigned c = funnel(w1, w0, 2);
            unsigned f;
            if constexpr (M == 0) f = c;
            else f = median_word<M>(w0, w1);
            if constexpr (MED < 0 && M != 0) {
                if (mixed) {
                    // each pixel takes F or E as its region's flag says; the
                    // word's rows cross at most one region boundary, at bit d
                    const int R = a.region, yr = y0 + wb, ry = yr / R;
                    const int d = (ry + 1) * R - yr;
                    const unsigned nxt = d >= 32 ? 0u : ~0u << d;
                    const int *fl = a.med_flags + (long long)ry * a.reg_gx + rx;
                    const unsigned s0 = fl[0] ? ~0u : 0u;
                    const unsigned s1 = (nxt != 0u && (ry + 1) * R < H) ? (fl[a.reg_gx] ? ~0u : 0u) : 0u;
                    const unsigned sel = (s0 & ~nxt) | (s1 & nxt);
                    f = (f & sel) | (c & ~sel);
                }
            }
            const unsigned rm = (n >= 32 ? ~0u : (1u << n) - 1u) & outm;
            ecnt += __popc(c & rm);
            fcnt += __popc(f & rm);
            // a wave-uniform row address plus the lane's column
            GlobalU8 *orow = (GlobalU8 *)(obase + (long long)(y0 + wb) * opitch);
            if (outc) {
#pragma unroll 8
                for (int k = 0; k < n; ++k) {
                    orow[(unsigned)xc] = (uint8_t)__builtin_amdgcn_ubfe(f, k, 1);
                    orow += opitch;
                }
            }
            elo = ehi;
            ehi = 0;
            wb += 32;
        };
        auto step = [&](const int si, const ZT &zv, auto clamp) __attribute__((always_inline)) {
            constexpr bool C = decltype(clamp)::value;
            double zn[2];
            ZStore<Acc>::get(zv, zn[0], zn[1]);
#pragma unroll
            for (int j = 0; j < 2; ++j) {   // row sums of the row just read (columns clamped by the loads)
                const double zl = from_left(zn[j]), zr = from_right(zn[j]);
                double hs, hq;
                dev_row(zl, zn[j], zr, hs, hq);
#pragma unroll
                for (int k = 0; k < NR - 1; ++k) {
                    Zs[j][k] = Zs[j][k + 1];
                    Zq[j][k] = Zq[j][k + 1];
                }
                Zs[j][NR - 1] = hs;
                Zq[j][NR - 1] = hq;
                if constexpr (S5) {
                    double ws, wq;
                    dev_row5(from_left(zl), from_right(zr), hs, hq, ws, wq);
#pragma unroll
                    for (int k = 0; k < NR - 1; ++k) {
                        Ws[j][k] = Ws[j][k + 1];
                        Wq[j][k] = Wq[j][k + 1];
                    }
                    Ws[j][NR - 1] = ws;
                    Wq[j][NR - 1] = wq;
                }
            }
            if constexpr (!C && MED >= 0) {
                // Interior strips: E as a sign bit.  dev > thr exactly when
                // thr - dev < 0 (finite values; their difference is 0 only
                // when they are equal, and then +0), so bit 31 of the high
                // word of thr - dev is E_j, and the words combine by AND
                // (the 5x5 stage) and OR (the two masks) before the bit is
                // moved into place: no lane masks and selects per row.  (Not
                // in the gated kernels, which hold two tile forms and would
                // lose occupancy to the registers this schedule takes.)
                unsigned eb = 0;
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const double s3[3] = {Zs[j][WR - 1], Zs[j][WR], Zs[j][WR + 1]};
                    const double q3[3] = {Zq[j][WR - 1], Zq[j][WR], Zq[j][WR + 1]};
                    unsigned e = (unsigned)__double2hiint((j == 0 ? thr72_0 : thr72_1) - dev_72var(s3, q3));
                    if constexpr (S5)
                        e &= (unsigned)__double2hiint((j == 0 ? thr600_0 : thr600_1) - dev_600var(Ws[j], Wq[j]));
                    eb |= e;
                }
                if (si >= 2 * WR) {
                    const int p = si - 2 * WR - wb;   // its bit in elo:ehi (wave-uniform)
                    const unsigned mlo = p < 32 ? 1u << p : 0u, mhi = p >= 32 ? 1u << (p - 32) : 0u;
                    const unsigned spread = (unsigned)((int)eb >> 31);   // E ? ~0 : 0
                    elo |= spread & mlo;
                    ehi |= spread & mhi;
                }
                return;
            }
            bool ej = false;
#pragma unroll
            for (int j = 0; j < 2; ++j) {   // deviations of Z around the middle row of the ring
                const double s3[3] = {Zs[j][WR - 1], Zs[j][WR], Zs[j][WR + 1]};
                const double q3[3] = {Zq[j][WR - 1], Zq[j][WR], Zq[j][WR + 1]};
                bool e = dev_72var(s3, q3) > (j == 0 ? thr72_0 : thr72_1);
                if constexpr (S5) e = e && (dev_600var(Ws[j], Wq[j]) > (j == 0 ? thr600_0 : thr600_1));
                ej = ej || e;
            }
            if (si >= 2 * WR) {
                const int y = y0 - HL - WR + si;   // the E row
                if constexpr (C) {           // rows below the image repeat row H - 1
                    if (y > H - 1) ej = last;
                    last = ej;
                }
                const int p = si - 2 * WR - wb;   // its bit in elo:ehi
                const unsigned mlo = p < 32 ? 1u << p : 0u, mhi = p >= 32 ? 1u << (p - 32) : 0u;
                const unsigned em = ej ? ~0u : 0u;
                elo |= em & mlo;
                ehi |= em & mhi;
                if constexpr (C) {           // rows above the image repeat row 0 (y0 = 0, bits 0 .. 2)
                    if (y == 0) elo = em & 7u;
                }
            }
        };
        auto run = [&](auto clamp) __attribute__((always_inline)) {
            // The last 2 HL rows this tile reads are the first ones the tile
            // below it reads: they are loaded first, so that the two tiles,
            // dispatched close together on one XCD, read them at about the
            // same time and the second read finds them in the L2.
            ZT tail[2 * HL];
#pragma unroll
            for (int k = 0; k < 2 * HL; ++k) {
                const int row = min(max(y0 + Rv - HL + k, 0), H - 1);
                tail[k] = zcol[(long long)row * W];
            }
            // full groups unrolled (loads first, the ring rotates by
            // renaming), the rest one step at a time, then the tail rows
            int si0 = 0;
            for (; si0 + G <= Rv; si0 += G) {
                ZT q[G];
#pragma unroll
                for (int k = 0; k < G; ++k) {
                    const int row = min(max(y0 - HL + si0 + k, 0), H - 1);
                    q[k] = zcol[(long long)row * W];
                }
#pragma unroll
                for (int k = 0; k < G; ++k) step(si0 + k, q[k], clamp);
                // E bits wb .. wb + 35 present: the word's 32 output rows are final
                if (si0 + G - 2 * WR - wb >= 36) emit(32);
            }
            for (; si0 < Rv; ++si0) {
                const int row = min(max(y0 - HL + si0, 0), H - 1);
                step(si0, zcol[(long long)row * W], clamp);
            }
            // (at most 35 + G - 1 + 2 HL < 64 E bits are pending here)
#pragma unroll
            for (int k = 0; k < 2 * HL; ++k) step(Rv + k, tail[k], clamp);
        };
        // the E rows y0-2 .. y0+Rv+1 the output uses lie inside the image:
        // no row clamping of the extracted bits
        if (y0 - 2 >= 0 && y0 + Rv + 1 <= H - 1) run(bool_c<false>{});
        else run(bool_c<true>{});
        while (wb < Rv) emit(min(32, Rv - wb));

        const int w = threadIdx.x / kWave;
        const int es = wave_sum((int)ecnt), fs = wave_sum((int)fcnt);
        if (lane == 0) {
            redc[0][w] = es;
            redc[1][w] = fs;
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
            tile(item, int_c<MED>{}, false);
        } else {   // gated: the median of each image (or region) as its flag says
            const int image = a.L.nimg == 1 ? 0 : a.L.owner2[item];
            int flag;
            bool mixed = false;
            if (a.region > 0) {
                // a tile inside one region takes that region's flag as a whole
                const ImageJob J = job_of(a.L, image);
                const int t = item - J.base2, tx = t % J.tiles_x2, ty = t / J.tiles_x2;
                const int x0 = tx * TW, y0 = ty * a.rows;
                const int x1 = min(x0 + TW, (int)J.img.W) - 1, y1 = min(y0 + a.rows, (int)J.img.H) - 1;
                const int R = a.region;
                mixed = x0 / R != x1 / R || y0 / R != y1 / R;
                flag = a.med_flags[(y0 / R) * a.reg_gx + x0 / R];
            } else {
                flag = a.med_flags[image];
            }
            if (mixed || flag) tile(item, int_c<-MED>{}, mixed);
            else tile(item, int_c<0>{}, false);
        }
    });
}

// One further level of the median cascade: reads a 0/1 map (clamp-to-edge
// rows and columns, which is how every level reads its input), collects
// each lane's column in words as pass 2 does, and writes the hybrid median
// (or, for an image the gate leaves unsmoothed, the map itself).
template <int HL, int M>
__global__ __launch_bounds__(256) void median_level_kernel(LevelArgs a) {
    __shared__ int redc[8];
    constexpr int OW = kWave - 2 * HL, TW = tile_out_width(HL);
    constexpr int G = 6;
    const int item = blockIdx.x;
    const int image = a.L.nimg == 1 ? 0 : a.L.owner2[item];
    const ImageJob J = job_of(a.L, image);
    const int H = (int)J.img.H, W = (int)J.img.W;
    const int tile = item - J.base2, tx = tile % J.tiles_x2, ty = tile / J.tiles_x2;
    const int x0 = tx * TW, y0 = ty * a.rows, Rv = min(a.rows, H - y0);
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int xc = x0 + wave * OW - HL + lane;
    const bool outc = lane >= HL && lane < HL + OW && xc < W;
    const unsigned outm = outc ? ~0u : 0u;
    const bool copy = a.med_flags && !a.med_flags[image];
    uint8_t *const scr = a.scratch + J.zoff;
    const uint8_t *const src = a.from_scratch ? scr : J.out;
    uint8_t *const dst = a.from_scratch ? J.out : scr;
    const long long spitch = a.from_scratch ? (long long)W : J.out_pitch;
    const long long dpitch = a.from_scratch ? J.out_pitch : (long long)W;
    const uint8_t *const scol = src + min(max(xc, 0), W - 1);

    // bit k of elo (of ehi): input row y0 - 2 + wb + k (+ 32)
    unsigned elo = 0, ehi = 0, fcnt = 0;
    int wb = 0;
    const int nrows = Rv + 4;   // input rows y0 - 2 .. y0 + Rv + 1
    auto emit = [&](const int n) __attribute__((always_inline)) {
        unsigned f = funnel(ehi, elo, 2);
        if (!copy) f = M == 3 ? median_word<3>(elo, ehi) : median_word<5>(elo, ehi);
        fcnt += __popc(f & (n >= 32 ? ~0u : (1u << n) - 1u) & outm);
        GlobalU8 *orow = (GlobalU8 *)(dst + (long long)(y0 + wb) * dpitch);
        if (outc) {
#pragma unroll 8
            for (int k = 0; k < n; ++k) {
                orow[(unsigned)xc] = (uint8_t)__builtin_amdgcn_ubfe(f, k, 1);
                orow += dpitch;
            }
        }
        elo = ehi;
        ehi = 0;
        wb += 32;
    };
    auto put = [&](const int b, const uint8_t v) __attribute__((always_inline)) {
        const int p = b - wb;
        const unsigned m = v != 0 ? ~0u : 0u;
        elo |= m & (p < 32 ? 1u << p : 0u);
        ehi |= m & (p >= 32 ? 1u << (p - 32) : 0u);
    };
    int b0 = 0;
    for (; b0 + G <= nrows; b0 += G) {
        uint8_t q[G];
#pragma unroll
        for (int k = 0; k < G; ++k) q[k] = scol[(long long)min(max(y0 - 2 + b0 + k, 0), H - 1) * spitch];
#pragma unroll
        for (int k = 0; k < G; ++k) put(b0 + k, q[k]);
        if (b0 + G - wb >= 36) emit(32);   // rows wb .. wb + 35 present
    }
    for (; b0 < nrows; ++b0) put(b0, scol[(long long)min(max(y0 - 2 + b0, 0), H - 1) * spitch]);
    while (wb < Rv) emit(min(32, Rv - wb));

    if (a.counts) {
        const int fs = wave_sum((int)fcnt);
        if (lane == 0) redc[threadIdx.x / kWave] = fs;
        __syncthreads();
        if (threadIdx.x == 0) {
            int t = 0;
            for (int k = 0; k < (int)(blockDim.x / kWave); ++k) t += redc[k];
            a.counts[(long long)item * 2 + 1] = t;
        }
    }
}

template <class Acc, int MED, bool S5>
hipError_t p2z5(const Pass2Args<typename AccOps<Acc>::Taps> &a, int grid, hipStream_t s, int *max_grid) {
    constexpr bool CAN_LOOP = MED >= 0;   // gated variants run one tile per workgroup
    if (max_grid) return occupancy(pass2z_kernel<Acc, MED, CAN_LOOP, S5>, 0, max_grid);
    if (!CAN_LOOP || grid >= a.L.total2)
        hipLaunchKernelGGL((pass2z_kernel<Acc, MED, false, S5>), dim3(a.L.total2), dim3(kTileWaves * kWave), 0, s, a);
    else
        hipLaunchKernelGGL((pass2z_kernel<Acc, MED, CAN_LOOP, S5>), dim3(grid), dim3(kTileWaves * kWave), 0, s, a);
    return hipGetLastError();
}
template <class Acc, int MED>
hipError_t p2z(const Pass2Args<typename AccOps<Acc>::Taps> &a, int grid, hipStream_t s, int *max_grid) {
    return a.std5 ? p2z5<Acc, MED, true>(a, grid, s, max_grid) : p2z5<Acc, MED, false>(a, grid, s, max_grid);
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
hipError_t launch_median_level(const LevelArgs &a, int halo, hipStream_t s) {
    const dim3 grid(a.L.total2), block(kTileWaves * kWave);
    if (halo == kHalo2Z5) {
        if (a.median_size == 3) hipLaunchKernelGGL((kern::median_level_kernel<kHalo2Z5, 3>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((kern::median_level_kernel<kHalo2Z5, 5>), grid, block, 0, s, a);
    } else {
        if (a.median_size == 3) hipLaunchKernelGGL((kern::median_level_kernel<kHalo2Z, 3>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((kern::median_level_kernel<kHalo2Z, 5>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace logfx
