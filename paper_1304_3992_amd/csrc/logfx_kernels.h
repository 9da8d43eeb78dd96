// HIP kernels of liblogfx for gfx950 (CDNA4, wave64).
//
// The pipeline (Tejaswi et al., arXiv:1304.3992, Sec. 4.1):
//   L_j = LoG_j * I (eq. (1) masks), Z_j = zero-crossing strength of L_j
//   (Sec. 3.2), E_j = [3x3 deviation of Z_j > T_j] (eq. (2)), E = E_1 | E_2,
//   F = hybrid_median(E) (Sec. 3.4).
// T_j depends on the global deviation of Z_j, a grid-wide quantity, so the
// work runs as   pass 1 (LoG, Z, per-tile sums; by default the pair
// (Z_1, Z_2) of every pixel stored to HBM) -> finalize (T_j) -> pass 2.
// Pass 2 normally reads the stored pairs (pass2z_kernel, in
// logfx_pass2z.hip: deviation, OR and the median on per-lane column words);
// the recompute form below (pass2_kernel) is the fallback when the pair
// memory cannot be had: it evaluates the LoG and Z again with a wider halo
// and takes the median on 64-bit wave-row ballots.
//
// Work decomposition of the image-reading passes.  A workgroup owns an
// output tile of kTileWaves wave-wide column strips side by side, `rows`
// rows tall; the input tile plus halo is staged once in LDS as u16 with
// clamp-to-edge coordinates.  Each lane owns one column and walks down the
// rows, keeping a ring of 2R+1 rows of horizontal pair sums in registers
// (32-bit, or packed 16-bit pairs in the integer path's packed form).
// Horizontal neighbours of later stages come from the adjacent lanes (DPP
// wave shifts on the vector ALU; lanes at the image border take their own
// value).
//
// Exactness.  Mask taps are integers k on a power-of-two grid, and the LoG
// is evaluated on D4 orbit sums of pixels, L = sum_o k_o * O_o, or in the
// packed form on the row-pair sums v(d, c) that make up the orbits, two
// taps per dot product.  Every sum is exact (int32 when
// sum|k| (2^bits - 1) < 2^30, else FP64 below 2^52), so L and Z agree bit
// for bit with any exact evaluation.
#pragma once
#include "logfx_internal.h"
#include "logfx_bits.h"

#include <type_traits>

namespace logfx {
namespace kern {

// ----------------------------------------------------------------- helpers
__device__ inline long long clampll(long long v, long long lo, long long hi) {
    return v < lo ? lo : (v > hi ? hi : v);
}

// Values of the lanes to the left (column x - 1) and right (x + 1), by DPP
// wave shifts on the vector ALU.  Lanes 0 and 63 receive 0 (they are halo
// lanes whose results are never used; no copy of the source is needed).
// At the image border the neighbour is clamped to the lane itself when the
// tile touches a border (EDGE); interior tiles skip the test.
__device__ inline int from_left(int v) { return __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true); }
__device__ inline int from_right(int v) { return __builtin_amdgcn_mov_dpp(v, 0x130, 0xf, 0xf, true); }
__device__ inline unsigned from_left(unsigned v) { return (unsigned)from_left((int)v); }
__device__ inline unsigned from_right(unsigned v) { return (unsigned)from_right((int)v); }
__device__ inline double from_left(double v) {
    return __hiloint2double(from_left(__double2hiint(v)), from_left(__double2loint(v)));
}
__device__ inline double from_right(double v) {
    return __hiloint2double(from_right(__double2hiint(v)), from_right(__double2loint(v)));
}
template <bool EDGE, class T>
__device__ inline void neighbours(T v, bool clampL, bool clampR, T &l, T &r) {
    l = from_left(v);
    r = from_right(v);
    if constexpr (EDGE) {
        l = clampL ? v : l;
        r = clampR ? v : r;
    }
}

// Accumulator policies: exact int32 or exact FP64 LoG sums.
template <class Acc> struct AccOps;
template <> struct AccOps<int> {
    using Taps = OrbitTapsI;
    template <class A> static __device__ int thr(const A &a, int j) { return a.zc_thr_i[j]; }
    // v_mad_i32_i24 on the raw tap register: both operands fit 24-bit signed
    // (|k| < 2^23 is checked on the host, o < 2^20), so no sign-extended
    // copies of the taps need to be kept alive.
    static __device__ int mac(int k, int o, int acc) {
        int r;
        asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "s"(k), "v"(o), "v"(acc));
        return r;
    }
    static __device__ double to_d(int v) { return (double)v; }
};
template <> struct AccOps<double> {
    using Taps = OrbitTapsD;
    template <class A> static __device__ double thr(const A &a, int j) { return a.zc_thr[j]; }
    static __device__ double mac(double k, int o, double acc) { return __fma_rn(k, (double)o, acc); }
    static __device__ double to_d(double v) { return v; }
};

// One row of horizontal pair sums at the lane's column: h[0] = I(x),
// h[j] = I(x - j) + I(x + j).
template <int RB>
__device__ inline void load_hrow(const uint16_t *p, int (&h)[RB + 1]) {
    h[0] = p[0];
#pragma unroll
    for (int j = 1; j <= RB; ++j) h[j] = (int)p[-j] + (int)p[j];
}

// Both LoG responses of the centre row of the ring (ring row RB).  Orbit
// (i, j), i >= j, is the set of offsets {(+-i, +-j), (+-j, +-i)}; its pixel
// sum is assembled from pair sums of the rows centre +- i and centre +- j.
template <class Acc, int RA, int RB>
__device__ inline void log_pair(const int (&h)[2 * RB + 1][RB + 1],
                                const typename AccOps<Acc>::Taps &t, Acc (&out)[2]) {
    Acc l0 = 0, l1 = 0;
#pragma unroll
    for (int i = 0; i <= RB; ++i) {
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            int o;
            if (i == 0) o = h[RB][0];
            else if (j == 0) o = h[RB][i] + h[RB - i][0] + h[RB + i][0];
            else if (i == j) o = h[RB - i][i] + h[RB + i][i];
            else o = h[RB - i][j] + h[RB + i][j] + h[RB - j][i] + h[RB + j][i];
            const int idx = orbit_index(i, j);
            if (i <= RA) l0 = AccOps<Acc>::mac(t.k[0][idx], o, l0);
            l1 = AccOps<Acc>::mac(t.k[1][idx], o, l1);
        }
    }
    out[0] = l0;
    out[1] = l1;
}

// Packed integer form (kP1Packed): pairs of 16-bit sums in one VGPR, the
// layout the taps' pk words describe.
typedef short pk2 __attribute__((ext_vector_type(2)));
__device__ inline pk2 as_pk2(unsigned v) { return __builtin_bit_cast(pk2, v); }
__device__ inline unsigned as_u32(pk2 v) { return __builtin_bit_cast(unsigned, v); }
__host__ __device__ constexpr int pk_words(int r) { return 1 + (r + 1) / 2; }

// (x.lo + y.hi, x.hi + y.lo): one v_pk_add_u16 with the halves of y swapped
// by its operand selection
__device__ inline pk2 add_swapped(unsigned x, unsigned y) {
    unsigned r;
    asm("v_pk_add_u16 %0, %1, %2 op_sel:[0,1] op_sel_hi:[1,0]" : "=v"(r) : "v"(x), "v"(y));
    return as_pk2(r);
}

// k * (low 16 bits of w), the 16 bits taken by the operand selection
__device__ inline int mul_lo16(int k, pk2 w) {
    int r;
    asm("v_mul_i32_i24_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:WORD_0"
        : "=v"(r) : "s"(k), "v"(as_u32(w)));
    return r;
}

// One row of pair sums at the lane's column, packed: g[0] = (I(x), I(x + 1))
// (the high half has zero taps), g[1] = (h_1, h_2), g[2] = (h_3, h_4),
// h_c = I(x - c) + I(x + c).  One unaligned 16-byte LDS read gives
// I(x - 4) .. I(x + 3) and one 2-byte read I(x + 4); the pairs (I1, I2)
// and (I3, I4) come from funnel shifts.  (Two 16-byte reads, at x - 4 and
// x - 3, spare the shifts but measured 35 % slower: the LDS, not the VALU,
// then bounds the kernel.)  For every mask radius these columns lie inside
// the staged row (its leading alignment columns and trailing padding hold
// them).
// The row's LDS words, read apart from their use so that the row loop can
// issue them a step ahead.
typedef unsigned RowV4 __attribute__((ext_vector_type(4), aligned(2)));
struct RowWords {
    RowV4 a;       // (I-4, I-3) (I-2, I-1) (I0, I1) (I2, I3)
    unsigned i4;   // I4 (radius 3 and 4)
};
template <int RB>
__device__ inline RowWords read_hrow_pk(const uint16_t *p) {
    RowWords w;
    w.a = *(const RowV4 *)(p - 4);
    w.i4 = pk_words(RB) > 2 ? p[4] : 0u;
    return w;
}
template <int RB>
__device__ inline void unpack_hrow_pk(const RowWords &w, pk2 (&g)[pk_words(RB)]) {
    g[0] = as_pk2(w.a.z);
    g[1] = add_swapped(__builtin_amdgcn_alignbit(w.a.w, w.a.z, 16), w.a.y);   // (I1, I2) + (I-1, I-2)
    if constexpr (pk_words(RB) > 2)
        g[2] = add_swapped(__builtin_amdgcn_alignbit(w.i4, w.a.w, 16), w.a.x);   // (I3, I4) + (I-3, I-4)
}
template <int RB>
__device__ inline void load_hrow_pk(const uint16_t *p, pk2 (&g)[pk_words(RB)]) {
    unpack_hrow_pk<RB>(read_hrow_pk<RB>(p), g);
}

// Both LoG responses of the centre row of the packed ring (ring row RB):
// the centre pixel times its 32-bit tap, then v(d, .) of the row pair at
// +-d by packed adds and two taps per v_dot2_i32_i16.
template <int RA, int RB>
__device__ inline void log_pair_pk(const pk2 (&g)[2 * RB + 1][pk_words(RB)], const OrbitTapsI &t, int (&out)[2]) {
    int l0 = mul_lo16(t.k[0][0], g[RB][0]);
    int l1 = mul_lo16(t.k[1][0], g[RB][0]);
#pragma unroll
    for (int d = 0; d <= RB; ++d) {
#pragma unroll
        for (int m = d == 0 ? 1 : 0; m < pk_words(RB); ++m) {
            const pk2 v = d == 0 ? g[RB][m] : g[RB - d][m] + g[RB + d][m];
            l1 = __builtin_amdgcn_sdot2(v, as_pk2(t.pk[1][d * kPkPerRow + m]), l1, false);
            if (d <= RA && m < pk_words(RA))
                l0 = __builtin_amdgcn_sdot2(v, as_pk2(t.pk[0][d * kPkPerRow + m]), l0, false);
        }
    }
    out[0] = l0;
    out[1] = l1;
}

// Opposite strict signs of p and q: the exact 64-bit product p q is
// negative, i.e. its high word is.  (Written without min / max, so that the
// crossing rule shares none with it and takes its five-value extremes in
// two three-input operations; the compiler keeps this test in the branch
// taken only when the wave has a zero pixel.)
__device__ inline bool opposite(int p, int q) { return __mulhi(p, q) < 0; }
__device__ inline bool opposite(double p, double q) { return p * q < 0.0; }

// Zero-crossing strength (Sec. 3.2) of centre a with neighbours up, dn, lf,
// rt, in grid units; returns the strength if a is a crossing stronger than
// thr, else 0.  For a < 0 the pair (a, q) with q > 0 marks a iff
// |a| <= |q|, i.e. a + q >= 0 (ties go to the negative pixel); for a > 0 it
// marks a iff a + q < 0.  The largest / smallest neighbour decides "some
// neighbour" at once.  A zero centre is a crossing when its left/right or
// up/down neighbours have opposite signs; that test only runs when some
// lane of the wave holds a zero.  Written without short-circuit logic so
// that it compiles to straight-line code.
// keep: an extra condition folded into the selection (0 where false).
template <class Acc, class Thr>
__device__ inline Acc zc_value(Acc a, Acc up, Acc dn, Acc lf, Acc rt, Thr thr, bool keep = true) {
    // hi / lo: largest / smallest of the five values.  For a < 0, a + hi >= 0
    // holds iff some neighbour reaches -a (a itself cannot), i.e. iff
    // a + max(neighbours) >= 0; for a > 0 likewise with lo.
    const Acc hi = max(max(max(max(up, dn), lf), rt), a);
    const Acc lo = min(min(min(min(up, dn), lf), rt), a);
    bool is;
    if constexpr (std::is_same<Acc, int>::value) {
        // b = a + hi for a <= 0, a + lo for a > 0 (exact: |L| < 2^30); a
        // crossing iff b and a differ in sign bit.  For a = 0, b = hi >= 0.
        const int b = a + (a <= 0 ? hi : lo);
        is = (b ^ a) < 0;
    } else {
        is = ((a < 0) & (a + hi >= 0)) | ((a > 0) & (a + lo < 0));
    }
    const Acc c = hi - lo;   // exact: |L| < 2^30 (int) or 2^52 (FP64)
    const bool strong = (c > thr) & keep;
    Acc r = (is & strong) ? c : Acc(0);
    if (__ballot(a == 0)) {
        const bool z = (a == 0) & (opposite(lf, rt) | opposite(up, dn));
        r = (z & strong) ? c : r;
    }
    return r;
}
template <class Acc, class Thr>
__device__ inline double zc_strength(Acc a, Acc up, Acc dn, Acc lf, Acc rt, Thr thr) {
    return AccOps<Acc>::to_d(zc_value<Acc>(a, up, dn, lf, rt, thr));
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}
__device__ inline int wave_sum(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// ---- bit-sliced logic for the binary hybrid median ----
// Every bit of a word is one pixel.  In the wave-row form bit l of a row
// mask is the pixel of lane l and sh(e, d) moves column x + d to bit l.
template <int D>
__device__ inline uint64_t sh(uint64_t e) {
    if constexpr (D >= 0) return e >> D;
    else return e << (-D);
}
// Hybrid median of the wave rows e[0..4] (rows r-2 .. r+2) around row 2
// (M = 3 or 5); a wave row whose window holds no extracted pixel stays 0
// without the bit network.
template <int M>
__device__ inline uint64_t hybrid_median(const uint64_t (&e)[5]) {
    if ((e[0] | e[1] | e[2] | e[3] | e[4]) == 0) return 0;
    if constexpr (M == 3) {
        const uint64_t p[4] = {sh<-1>(e[2]), sh<1>(e[2]), e[1], e[3]};
        const uint64_t x[4] = {sh<-1>(e[1]), sh<1>(e[1]), sh<-1>(e[3]), sh<1>(e[3])};
        return hybrid_median_bits<3>(e[2], p, x);
    } else {
        const uint64_t p[8] = {sh<-2>(e[2]), sh<-1>(e[2]), sh<1>(e[2]), sh<2>(e[2]), e[0], e[1], e[3], e[4]};
        const uint64_t x[8] = {sh<-2>(e[0]), sh<2>(e[0]), sh<-1>(e[1]), sh<1>(e[1]),
                               sh<-1>(e[3]), sh<1>(e[3]), sh<-2>(e[4]), sh<2>(e[4])};
        return hybrid_median_bits<5>(e[2], p, x);
    }
}

// Row sums of the 3x3 deviation (eq. (2)) at one pixel: s = z_l + z + z_r
// and q = z_l^2 + z^2 + z_r^2 of the pixel's row, in a fixed FP64 order
// that every pass uses, so that the deviation test decides the same way.
__device__ inline void dev_row(double zl, double z, double zr, double &s, double &q) {
    s = (zl + z) + zr;
    q = __fma_rn(zr, zr, __fma_rn(zl, zl, z * z));
}
// 72 s^2 = 9 sum z^2 - (sum z)^2 over the three rows of the window.
__device__ inline double dev_72var(const double (&s)[3], const double (&q)[3]) {
    const double S = (s[0] + s[1]) + s[2];
    const double Q = (q[0] + q[1]) + q[2];
    return __fma_rn(-S, S, 9.0 * Q);
}

// Replicate the bit of the first / last in-image lane into the lanes that
// lie left / right of the image, so shifted reads see clamped columns.
__device__ inline uint64_t clamp_bits(uint64_t e, int lo, int hi) {
    if (lo > 0) {
        const uint64_t m = (1ull << lo) - 1;
        e = (e & ~m) | (((e >> lo) & 1ull) ? m : 0ull);
    }
    if (hi < kWave - 1) {
        const uint64_t m = ~((2ull << hi) - 1);
        e = (e & ~m) | (((e >> hi) & 1ull) ? m : 0ull);
    }
    return e;
}

// Eight pixels from element `at` of an image (u16 when `u16`, else u8
// widened to u16) at any pixel alignment: one 16- or 8-byte global load,
// which gfx950 serves under the HSA unaligned access mode.
__device__ inline uint4 load8(const void *data, long long at, bool u16) {
    typedef __attribute__((address_space(1))) const uint16_t GU16;
    typedef __attribute__((address_space(1))) const uint8_t GU8;
    typedef unsigned V4 __attribute__((ext_vector_type(4), aligned(2)));
    typedef unsigned V2 __attribute__((ext_vector_type(2), aligned(1)));
    typedef __attribute__((address_space(1))) const V4 GV4;
    typedef __attribute__((address_space(1))) const V2 GV2;
    if (u16) {
        const V4 q = *(GV4 *)((GU16 *)data + at);
        return make_uint4(q.x, q.y, q.z, q.w);
    }
    const V2 q = *(GV2 *)((GU8 *)data + at);
    return make_uint4(__builtin_amdgcn_perm(0u, q.x, 0x0c010c00u), __builtin_amdgcn_perm(0u, q.x, 0x0c030c02u),
                      __builtin_amdgcn_perm(0u, q.y, 0x0c010c00u), __builtin_amdgcn_perm(0u, q.y, 0x0c030c02u));
}

// ------------------------------------------------------------- strips
// Geometry shared by both passes.  A workgroup owns a tile of kTileWaves strips
// side by side; each wave's 64 lanes cover image columns base .. base+63,
// of which lanes HL .. 63-HL are output columns.  Everything but the lane's
// own column is wave-uniform and lives in scalar registers.
template <int HL, int RB>
struct Strip {
    static constexpr int OW = kWave - 2 * HL;
    static constexpr int TW = tile_out_width(HL);         // output columns per tile
    static constexpr int OFF = tile_lds_offset(HL, RB);   // LDS column of image column x0-HL-RB
    static constexpr int stride = tile_lds_stride(HL, RB);  // LDS row pitch (u16), 8-multiple
    int H, W, x0, y0, Rv, RH;
    int lane, base, xc, lc;
    bool outc, clampL, clampR;   // output column; left / right neighbour is the lane itself

    __device__ Strip(const ImageDesc &img, int tile, int tiles_x, int rows) {
        H = (int)img.H;
        W = (int)img.W;
        const int tx = tile % tiles_x, ty = tile / tiles_x;
        x0 = tx * TW;
        y0 = ty * rows;
        Rv = min(rows, H - y0);
        RH = Rv + 2 * HL + 2 * RB;
        lane = threadIdx.x & (kWave - 1);
        // the wave index is uniform across the wave: keep it (and all that
        // derives from it) in scalar registers
        const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
        base = x0 + wave * OW - HL;
        xc = base + lane;
        lc = wave * OW + lane + RB + OFF;
        clampL = xc <= 0;
        clampR = xc >= W - 1;
        // held as one value, so that each use tests it once instead of
        // re-deriving the lane range
        int oc = lane >= HL && lane < HL + OW && xc < W;
        asm("v_mov_b32 %0, %1" : "=v"(oc) : "v"(oc));
        outc = oc != 0;
    }

    // Stage the input rows y0-HL-RB .. (RH rows) and columns from the
    // 8-aligned origin x0-HL-RB-OFF (stride columns) in LDS as u16, with
    // clamp-to-edge coordinates, in chunks of 8 pixels.  Chunks inside the
    // image are one load each (load8: any pixel alignment, so neither the
    // image's start nor its pitch need be aligned), 8 in flight per thread.
    // In tiles at the left or right border, the chunks that reach past it
    // (the first nl and the last CPR - nr of each row) are then read pixel
    // by pixel with clamped columns.  Consecutive threads take consecutive
    // chunks of a row (coalesced); chunk i of the tile starts at LDS element
    // 8 i (the LDS row pitch is CPR chunks).
    __device__ void fill(uint16_t *lds, const ImageDesc &img) const {
        constexpr int CPR = stride / 8;
        const int ry0 = y0 - HL - RB, rx0 = x0 - HL - RB - OFF;
        const int nch = RH * CPR;
        const int nt = blockDim.x;
        const long long pitch = img.pitch;
        const bool u16 = img.dtype == 1;
        // chunks nl .. nr-1 of a row lie inside the image columns
        const int nl = rx0 >= 0 ? 0 : min((-rx0 + 7) / 8, CPR);
        const int nr = max(nl, min(CPR, (W - rx0) / 8));
        for (int b = 0; b < nch; b += 8 * nt) {
            uint4 v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int i = b + k * nt + (int)threadIdx.x;
                const int row = i / CPR, ch = i - row * CPR;
                if (i < nch && ch >= nl && ch < nr) {
                    const long long at = (long long)min(max(ry0 + row, 0), H - 1) * pitch + rx0 + 8 * ch;
                    v[k] = load8(img.data, at, u16);
                }
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int i = b + k * nt + (int)threadIdx.x;
                const int row = i / CPR, ch = i - row * CPR;
                if (i < nch && ch >= nl && ch < nr) *(uint4 *)(lds + 8 * i) = v[k];
            }
        }
        const int nb = nl + CPR - nr;   // border chunks per row
        if (nb == 0) return;
        typedef __attribute__((address_space(1))) const uint16_t GU16;
        typedef __attribute__((address_space(1))) const uint8_t GU8;
        for (int e = (int)threadIdx.x; e < RH * nb; e += nt) {
            const int row = e / nb, j = e - row * nb;
            const int ch = j < nl ? j : nr + (j - nl);
            const long long at = (long long)min(max(ry0 + row, 0), H - 1) * pitch;
            const int c0 = rx0 + 8 * ch;
            unsigned p[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const long long o = at + min(max(c0 + q, 0), W - 1);
                p[q] = u16 ? (unsigned)((GU16 *)img.data)[o] : (unsigned)((GU8 *)img.data)[o];
            }
            *(uint4 *)(lds + 8 * (row * CPR + ch)) =
                make_uint4(p[0] | p[1] << 16, p[2] | p[3] << 16, p[4] | p[5] << 16, p[6] | p[7] << 16);
        }
    }
};

// Row rings keep clamp-to-edge rows: a row past the bottom of the image
// repeats the last image row, and when row 0 arrives it is copied over the
// rows above it.  Every stage can then read its ring without border tests.
// Strips that stay clear of the top and bottom rows skip the tests (CLAMP
// false).
template <bool CLAMP, class T, int N>
__device__ inline void ring_push(T (&ring)[N], T v, int row, int H) {
    if (CLAMP && row > H - 1) v = ring[N - 1];
#pragma unroll
    for (int k = 0; k < N - 1; ++k) ring[k] = ring[k + 1];
    ring[N - 1] = v;
    if (CLAMP && row == 0) {
#pragma unroll
        for (int k = 0; k < N - 1; ++k) ring[k] = v;
    }
}

template <bool B> using bool_c = std::integral_constant<bool, B>;
template <int V> using int_c = std::integral_constant<int, V>;

// ------------------------------------------------------------- work list
// Tiles of a launch are split into 8 contiguous shares, one per XCD
// (workgroups are dispatched round-robin over the XCDs), so neighbouring
// tiles, which share halo rows and columns, meet in the same L2.  The
// workgroups of an XCD stride through its share: one tile each when the
// grid has one workgroup per tile, several in a persistent launch.
// LOOP false: one workgroup per tile (grid = total), no loop in the code.
template <bool LOOP, class F>
__device__ inline void for_each_tile(int total, F &&f) {
    constexpr int X = 8;
    const int G = gridDim.x, b = blockIdx.x;
    const int x = b % X, l = b / X;
    const int start = x * (total / X) + min(x, total % X);
    if constexpr (!LOOP) {
        f(start + l);
    } else {
        const int len = total / X + (x < total % X);
        const int nx = G / X + (x < G % X);
        for (int i = l; i < len; i += nx) f(start + i);
    }
}

// acc + [z != 0] per lane, and the wave's lane mask of z != 0: one compare
// whose mask is the carry-in of one add.  (Written as C, the compiler keeps
// the compare's mask across the strength store's branch and rebuilds it as
// 0 / 1 in a register before adding.)
__device__ inline unsigned count_nonzero(unsigned acc, int z, uint64_t &mask) {
    unsigned r;
    uint64_t co;
    asm("v_cmp_ne_u32_e64 %1, 0, %3\n\tv_addc_co_u32 %0, %2, 0, %4, %1"
        : "=v"(r), "=&s"(mask), "=s"(co) : "v"(z), "v"(acc));
    return r;
}

__device__ inline ImageJob job_of(const Launch &L, int image) {
    return L.nimg == 1 ? L.one : L.jobs[image];
}


// Storage of the crossing-strength pair of a pixel between the passes: the
// integer path keeps the exact integer strengths as int32 pairs, the FP64
// path as double pairs (LoG grid units either way).
template <class Acc> struct ZStore;
template <> struct ZStore<int> {
    using T = int2;
    __device__ static T make(const int (&z)[2]) { return make_int2(z[0], z[1]); }
    __device__ static void get(const T &v, double &z0, double &z1) {
        z0 = (double)v.x;
        z1 = (double)v.y;
    }
};
template <> struct ZStore<double> {
    using T = double2;
    __device__ static T make(const double (&z)[2]) { return make_double2(z[0], z[1]); }
    __device__ static void get(const T &v, double &z0, double &z1) {
        z0 = v.x;
        z1 = v.y;
    }
};

// ------------------------------------------------------------- pass 1
// Occupancy: the integer path is held to 128 VGPRs (4 waves per SIMD, the
// LDS limit); the FP64 path keeps its registers.  Variants that need more
// run at fewer waves rather than spill.  No kernel here may spill vector
// registers (the build refuses one that does): the crossing test reads its
// neighbours from the adjacent lanes (DPP), and a spill reload that the
// compiler places under a partial execution mask (a store for the output
// lanes only) leaves the halo lanes' copies stale, which wrong neighbours
// then show at the wave borders.  Spills were also slower: a reload waits
// for every outstanding vector memory operation, the strength stores
// included.
template <class Acc> constexpr int kMinWaves = std::is_same<Acc, int>::value ? 4 : 1;
template <class Acc, int MODE, bool LOOP>
constexpr int kPass1Waves =
    !std::is_same<Acc, int>::value ? kMinWaves<Acc>
    : (MODE & kP1Maps) != 0 ? 2   // inspection only: room for the FP64 map writes
    : (MODE & kP1Packed) != 0 ? 4
    : (MODE & kP1Cells) != 0 || LOOP ? 3
    : kMinWaves<Acc>;
// The recomputing pass 2 (the fallback without stored strengths) keeps the
// LoG rings, the deviation rows and the median rows at once.
template <class Acc> constexpr int kPass2Waves = std::is_same<Acc, int>::value ? 2 : 1;

// MODE, a set of bits: 0 = statistics only; kP1Maps = also the FP64 maps
// of a single image; kP1Cells = also the per-cell sums of the gate
// features; kP1StoreZ = also the crossing-strength pair (Z_1, Z_2) of every
// pixel, for pass 2 to read instead of recomputing it.
template <class Acc, int RA, int RB, int MODE, bool LOOP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kPass1Waves<Acc, MODE, LOOP>))) void pass1_kernel(Pass1Args<typename AccOps<Acc>::Taps> a) {
    extern __shared__ uint16_t lds[];
    __shared__ double red[4][8];
    __shared__ long long redc[2][8];
    // cell sums of the current cell row, one slot per cell column a tile
    // touches (a.cell_slots of them), in the dynamic LDS after the tile: a
    // fixed array for the worst case (248 one-pixel cells) would push the
    // workgroup past a quarter of the CU's LDS
    unsigned *const cellv = reinterpret_cast<unsigned *>(lds + Strip<kHalo1, RB>::stride * (a.rows + 1 + 2 * kHalo1 + 2 * RB));
    unsigned *const cellc = cellv + a.cell_rows * a.cell_slots;
    constexpr int HL = kHalo1, P = 2 * RB + 1;
    // The step schedule below takes one halo row above and below the strip:
    // the crossing row r = t - 1 is an output row from the third step to the
    // last.  A wider halo would store rows outside the strip (and, at the
    // image's top and bottom, outside the strength map).
    static_assert(HL == 1, "pass 1 steps assume a one-row halo");

    for_each_tile<LOOP>(a.L.total1, [&](const int item) __attribute__((always_inline)) {
    const ImageJob J = job_of(a.L, a.L.nimg == 1 ? 0 : a.L.owner1[item]);
    const Strip<HL, RB> g(J.img, item - J.base1, J.tiles_x1, a.rows);
    // the fill at raised wave priority: its loads issue ahead of the other
    // workgroups' arithmetic on the SIMD, which shortens the wait at the
    // barrier (pass 1 about 2 % faster)
    __builtin_amdgcn_s_setprio(3);
    g.fill(lds, J.img);
    if constexpr ((MODE & kP1Cells) != 0) {
        for (int i = threadIdx.x; i < a.cell_rows * a.cell_slots; i += blockDim.x) cellv[i] = cellc[i] = 0;
    }
    __syncthreads();
    __builtin_amdgcn_s_setprio(0);

    // ring of pair-sum rows: 32-bit, or packed (kP1Packed)
    constexpr bool PK = (MODE & kP1Packed) != 0;
    static_assert(!PK || std::is_same<Acc, int>::value, "the packed form is integer only");
    int h[PK ? 1 : P][RB + 1];
    pk2 hp[PK ? P : 1][pk_words(RB)];
#pragma unroll
    for (int s = 0; s < P - 1; ++s) {
        if constexpr (PK) load_hrow_pk<RB>(lds + s * g.stride + g.lc, hp[s + 1]);
        else load_hrow<RB>(lds + s * g.stride + g.lc, h[s + 1]);
    }
    Acc L[2][3] = {{0, 0, 0}, {0, 0, 0}};   // rows t-2, t-1, t per mask
    double sz[2] = {0.0, 0.0}, sq[2] = {0.0, 0.0};
    int cnt[2] = {0, 0};
    const int nsteps = g.Rv + 2 * HL;
    const int t0 = g.y0 - HL;
    const uint16_t *lrow = lds + (2 * RB) * g.stride + g.lc;   // LDS row of step si
    // packed form: the words of the next step's row, read one step ahead
    // (the last step's read lands in the spare LDS row after the tile); the
    // cell-summing variants of the two widest radius pairs would spill the
    // five registers it holds and read each row in its step
    constexpr bool AHEAD = PK && ((MODE & kP1Cells) == 0 || RA + RB < 7);
    RowWords ahead{};
    if constexpr (AHEAD) ahead = read_hrow_pk<RB>(lrow);

    // Feature mode: the image is cut into CY x CX cells, CY = 2^cells_ly,
    // CX = 2^cells_lx (row r and column x belong to cell (r * CY / H,
    // x * CX / W)).
    // Each lane sums its pixel values and crossing indicators down its
    // column while the rows stay in one cell row.  At the end of a cell row
    // (or of the strip) the lanes add their sums into the tile's LDS slot of
    // that cell -- one slot per (cell row, cell column) the tile spans, so no
    // slot is reused within the tile and the row loop needs no barrier.
    // After the last row one thread per slot adds the slot to the image's
    // cell counters (integer atomics: exact and order-free).
    // The row loop keeps one scalar of this bookkeeping, fend (the strip
    // row that ends the current cell row); the rest is wave-uniform but held
    // in vector registers (fcy, the slot-row base fat) or recomputed after
    // the loop, so that the loop's scalar registers do not spill.
    auto cell_of = [](long long n, int cells, long long d) {
        // floor(n * cells / d) in FP64: exact, since n * cells < 2^53 and a
        // non-integer quotient lies at least 1/d from an integer
        return (int)floor((double)n * cells / (double)d);
    };
    unsigned fv = 0;            // value sum
    unsigned fc[2] = {0, 0};    // crossings of mask 1, of mask 2
    int fcy = 0, fat = 0;       // current cell row (vector register); its slot row's first slot
    int fslot = 0;              // the slot of the lane's cell column (output lanes)
    int fend = 0;               // the strip row that ends the current cell row
    const int flast = g.y0 + g.Rv - 1;
    // the last row of cell row cy: the first row of cy + 1, less one
    auto cell_end = [&](const long long cy) __attribute__((always_inline)) {
        return (int)((((cy + 1) * g.H + (1ll << a.cells_ly) - 1) >> a.cells_ly) - 1);
    };
    if constexpr ((MODE & kP1Cells) != 0) {
        const int CX = 1 << a.cells_lx, CY = 1 << a.cells_ly;
        const int fkey0 = cell_of(g.x0, CX, g.W);
        fslot = g.outc ? cell_of(g.xc, CX, g.W) - fkey0 : 0;
        const int fcy0 = cell_of(g.y0, CY, g.H);
        asm("v_mov_b32 %0, %1" : "=v"(fcy) : "v"(fcy0));
        fend = min(cell_end(fcy0), flast);
    }
    auto flush = [&](const int r) __attribute__((always_inline)) {
        if (g.outc && (fv | fc[0] | fc[1])) {
            const int at = fat + fslot;
            atomicAdd(&cellv[at], fv);
            atomicAdd(&cellc[at], fc[0] | fc[1] << 16);
        }
        fv = fc[0] = fc[1] = 0;
        // the cell row of row r + 1 (cells may be empty when H < cells):
        // the first c > fcy whose rows reach past r, by shifts only
        int cy = fcy + 1;
        while (cell_end(cy) < r + 1) ++cy;
        fat += (cy - fcy) * a.cell_slots;
        fcy = cy;
        // wave-uniform: the next flush row as a scalar
        fend = min(__builtin_amdgcn_readfirstlane(cell_end(cy)), flast);
    };

    // One step = one new input row.  Full groups of P steps are unrolled so
    // the register rings rotate by renaming; the last partial group runs
    // rolled.
    auto step = [&](const int si, auto clamp) __attribute__((always_inline)) {
        constexpr bool C = decltype(clamp)::value;
        Acc Ln[2];
        if constexpr (PK) {
#pragma unroll
            for (int s = 0; s < P - 1; ++s)
#pragma unroll
                for (int m = 0; m < pk_words(RB); ++m) hp[s][m] = hp[s + 1][m];
            if constexpr (AHEAD) {
                unpack_hrow_pk<RB>(ahead, hp[P - 1]);
                ahead = read_hrow_pk<RB>(lrow + g.stride);
            } else {
                load_hrow_pk<RB>(lrow, hp[P - 1]);
            }
            log_pair_pk<RA, RB>(hp, a.taps, Ln);
        } else {
#pragma unroll
            for (int s = 0; s < P - 1; ++s)
#pragma unroll
                for (int j = 0; j <= RB; ++j) h[s][j] = h[s + 1][j];
            load_hrow<RB>(lrow, h[P - 1]);
            log_pair<Acc, RA, RB>(h, a.taps, Ln);
        }
        lrow += g.stride;
        const int t = t0 + si;
        ring_push<C>(L[0], Ln[0], t, g.H);
        ring_push<C>(L[1], Ln[1], t, g.H);
        // zero crossings of row t - 1 (valid from the third step on)
        const int r = t - 1;
        const bool use = g.outc & (si >= 2);
        Acc zr[2];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const Acc c = L[j][1];
            Acc lf, rt;
            neighbours<C>(c, g.clampL, g.clampR, lf, rt);
            // the strength where this lane holds an output pixel of the strip, else 0
            zr[j] = zc_value<Acc>(c, L[j][0], L[j][2], lf, rt, AccOps<Acc>::thr(a, j), use);
            const double z = AccOps<Acc>::to_d(zr[j]);
            sz[j] += z;
            sq[j] = __fma_rn(z, z, sq[j]);
            if constexpr ((MODE & kP1Cells) != 0 && std::is_same<Acc, int>::value) {
                // the cell's crossing count and the wave's in one compare
                uint64_t nz;
                fc[j] = count_nonzero(fc[j], zr[j], nz);
                cnt[j] += __popcll(nz);   // wave-uniform
            } else {
                cnt[j] += __popcll(__ballot(zr[j] != Acc(0)));   // wave-uniform
                if constexpr ((MODE & kP1Cells) != 0) fc[j] += (unsigned)(zr[j] != Acc(0));
            }
            if constexpr ((MODE & kP1Maps) != 0) {
                if (use) {
                    const long long at = (long long)r * g.W + g.xc;
                    if (a.dbgL[j]) a.dbgL[j][at] = AccOps<Acc>::to_d(c) * a.unit[j];
                    if (a.dbgZ[j]) a.dbgZ[j][at] = z * a.unit[j];
                }
            }
        }
        if constexpr ((MODE & kP1StoreZ) != 0) {
            // the row's base is wave-uniform: scalar base + the lane's column
            typename ZStore<Acc>::T *zrow =
                static_cast<typename ZStore<Acc>::T *>(a.zmap) + (J.zoff + (long long)r * g.W);
            if (use) zrow[g.xc] = ZStore<Acc>::make(zr);
        }
        if constexpr ((MODE & kP1Cells) != 0) {
            // every lane accumulates; the halo rows before the strip are
            // dropped below and the non-output lanes at the flush
            // pixel (r, xc): the centre of ring row RB - 1
            if constexpr (PK) fv += as_u32(hp[RB - 1][0]) & 0xFFFFu;
            else fv += (unsigned)h[RB - 1][0];
            if (si < 2) fv = fc[0] = fc[1] = 0;
            else if (r == fend) flush(r);
        }
    };
    auto run = [&](auto clamp) __attribute__((always_inline)) {
        int si0 = 0;
        for (; si0 + P <= nsteps; si0 += P) {
#pragma unroll
            for (int ph = 0; ph < P; ++ph) step(si0 + ph, clamp);
        }
        for (; si0 < nsteps; ++si0) step(si0, clamp);
    };
    // interior tile: every row and column the strip touches lies strictly
    // inside the image, so no border test is needed
    const bool inner_x = g.x0 - HL >= 1 && g.x0 + Strip<HL, RB>::TW + HL <= g.W - 1;
    if (inner_x && t0 >= 1 && t0 + nsteps - 1 <= g.H - 1) run(bool_c<false>{});
    else run(bool_c<true>{});

    if constexpr ((MODE & kP1Cells) != 0) {
        // the tile's cell slots into the image's counters, one thread per slot
        __syncthreads();
        unsigned long long *fcells =
            a.cells + ((long long)(a.L.nimg == 1 ? 0 : a.L.owner1[item]) << (a.cells_lx + a.cells_ly + 1));
        const int CX = 1 << a.cells_lx, CY = 1 << a.cells_ly;
        const int fkey0 = cell_of(g.x0, CX, g.W);
        const int fslots = cell_of(min(g.x0 + Strip<HL, RB>::TW, g.W) - 1, CX, g.W) - fkey0 + 1;
        const int fcy0 = cell_of(g.y0, CY, g.H);
        const int fspan = cell_of(flast, CY, g.H) - fcy0 + 1;
        for (int i = threadIdx.x; i < fspan * fslots; i += blockDim.x) {
            const int cr = i / fslots, cc = i - cr * fslots;
            const unsigned v = cellv[cr * a.cell_slots + cc];
            const unsigned c = cellc[cr * a.cell_slots + cc];
            if (v | c) {
                unsigned long long *cell = fcells + ((long long)(fcy0 + cr) << a.cells_lx) + fkey0 + cc;
                atomicAdd(cell, (unsigned long long)v);
                atomicAdd(cell + (1ll << (a.cells_lx + a.cells_ly)),
                          (unsigned long long)(c & 0xFFFFu) | ((unsigned long long)(c >> 16) << 32));
            }
        }
    }

    // Deterministic per-tile reduction: fixed butterfly per wave, then the
    // waves in order.
    const int wave = threadIdx.x / kWave;
    double v[4] = {wave_sum(sz[0]), wave_sum(sz[1]), wave_sum(sq[0]), wave_sum(sq[1])};
    if (g.lane == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) red[k][wave] = v[k];
        redc[0][wave] = cnt[0];
        redc[1][wave] = cnt[1];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = blockDim.x / kWave;
        double s[4] = {0, 0, 0, 0};
        long long cc[2] = {0, 0};
        for (int w = 0; w < nw; ++w) {
#pragma unroll
            for (int k = 0; k < 4; ++k) s[k] += red[k][w];
            cc[0] += redc[0][w];
            cc[1] += redc[1][w];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) a.partials[(long long)item * 4 + k] = s[k];
        a.counts[(long long)item * 2 + 0] = cc[0];
        a.counts[(long long)item * 2 + 1] = cc[1];
    }
    __syncthreads();   // LDS and the reduction buffers are reused by the next tile
    });
}

// ------------------------------------------------------------- pass 2
// MED: 0 = no smoothing (output E), 3 or 5 = hybrid median window, -3 or
// -5 = that window on the images whose med_flags entry is set, none on the
// others (one kernel; the choice is uniform over a workgroup).
template <class Acc, int RA, int RB, int MED, bool LOOP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kPass2Waves<Acc>))) void pass2_kernel(Pass2Args<typename AccOps<Acc>::Taps> a) {
    extern __shared__ uint16_t lds[];
    __shared__ int redc[2][8];
    constexpr int HL = kHalo2, P = 2 * RB + 1;

    auto tile = [&](const int item, auto medc) __attribute__((always_inline)) {
    constexpr int M = decltype(medc)::value;
    const int image = a.L.nimg == 1 ? 0 : a.L.owner2[item];
    const ImageJob J = job_of(a.L, image);
    const Strip<HL, RB> g(J.img, item - J.base2, J.tiles_x2, a.rows);
    g.fill(lds, J.img);
    __syncthreads();

    const double thr72_0 = a.stats[image].thr72[0], thr72_1 = a.stats[image].thr72[1];
    // lanes of the first / last image column inside this wave (for the
    // bit-level clamping of the extracted map)
    const int lo_lane = g.base < 0 ? -g.base : 0;
    const int hi_lane = min(max(g.W - 1 - g.base, 0), kWave - 1);
    const uint64_t mybit = 1ull << g.lane;
    const uint64_t outmask = __ballot(g.outc);

    int h[P][RB + 1];
#pragma unroll
    for (int s = 0; s < P - 1; ++s) load_hrow<RB>(lds + s * g.stride + g.lc, h[s + 1]);
    Acc L[2][3] = {{0, 0, 0}, {0, 0, 0}};        // rows t-2, t-1, t
    double Zs[2][3] = {{0, 0, 0}, {0, 0, 0}};    // deviation row sums, rows t-3, t-2, t-1
    double Zq[2][3] = {{0, 0, 0}, {0, 0, 0}};
    uint64_t e[5] = {0, 0, 0, 0, 0};             // rows t-6 .. t-2
    int ecnt = 0, fcnt = 0;
    const int nsteps = g.Rv + 2 * HL;
    const int t0 = g.y0 - HL;
    // output row t - 4 of step si; advanced by one row per step.  The pitch
    // is moved to a vector register so the per-step offsets are not
    // materialised as scalar constants.
    uint8_t *orow = J.out + (long long)(t0 - 4) * J.out_pitch + g.xc;
    long long opitch;
    asm("v_mov_b64 %0, %1" : "=v"(opitch) : "s"(J.out_pitch));
    const uint16_t *lrow = lds + (2 * RB) * g.stride + g.lc;   // LDS row of step si

    auto step = [&](const int si, auto clamp) __attribute__((always_inline)) {
        constexpr bool C = decltype(clamp)::value;
#pragma unroll
        for (int s = 0; s < P - 1; ++s)
#pragma unroll
            for (int j = 0; j <= RB; ++j) h[s][j] = h[s + 1][j];
        load_hrow<RB>(lrow, h[P - 1]);
        lrow += g.stride;
        const int t = t0 + si;
        Acc Ln[2];
        log_pair<Acc, RA, RB>(h, a.taps, Ln);
        ring_push<C>(L[0], Ln[0], t, g.H);
        ring_push<C>(L[1], Ln[1], t, g.H);
        // The later stages run from the first step on; what they compute
        // before their inputs are valid leaves the rings before any output
        // uses it.  Only the output is guarded.
#pragma unroll
        for (int j = 0; j < 2; ++j) {   // zero-crossing strength of row t - 1 and its row sums
            const Acc c = L[j][1];
            Acc lf, rt;
            neighbours<C>(c, g.clampL, g.clampR, lf, rt);
            const double z = zc_strength<Acc>(c, L[j][0], L[j][2], lf, rt, AccOps<Acc>::thr(a, j));
            double zl, zr, hs, hq;
            neighbours<C>(z, g.clampL, g.clampR, zl, zr);
            dev_row(zl, z, zr, hs, hq);
            ring_push<C>(Zs[j], hs, t - 1, g.H);
            ring_push<C>(Zq[j], hq, t - 1, g.H);
        }
        bool ej = false;
#pragma unroll
        for (int j = 0; j < 2; ++j)     // extraction of row t - 2: 3x3 deviation of Z
            ej = ej || (dev_72var(Zs[j], Zq[j]) > (j == 0 ? thr72_0 : thr72_1));
        ring_push<C>(e, clamp_bits(__ballot(ej), lo_lane, hi_lane), t - 2, g.H);
        // output row t - 4 (from the ninth step on)
        uint64_t f;
        if constexpr (M == 0) f = e[2];
        else f = hybrid_median<M>(e);
        if (si >= 8) {
            if (g.outc) *orow = (uint8_t)((f & mybit) != 0);
            fcnt += __popcll(f & outmask);       // wave-uniform counts
            ecnt += __popcll(e[2] & outmask);
        }
        orow += opitch;
    };
    auto run = [&](auto clamp) __attribute__((always_inline)) {
        int si0 = 0;
        for (; si0 + P <= nsteps; si0 += P) {
#pragma unroll
            for (int ph = 0; ph < P; ++ph) step(si0 + ph, clamp);
        }
        for (; si0 < nsteps; ++si0) step(si0, clamp);
    };
    // interior tile: rows t-2 .. t of every step and every column of the
    // strip lie strictly inside the image, so no border test is needed
    const bool inner_x = g.x0 - HL >= 1 && g.x0 + Strip<HL, RB>::TW + HL <= g.W - 1;
    if (inner_x && t0 - 2 >= 1 && t0 + nsteps - 1 <= g.H - 1) run(bool_c<false>{});
    else run(bool_c<true>{});

    const int wave = threadIdx.x / kWave;
    if (g.lane == 0) {
        redc[0][wave] = ecnt;
        redc[1][wave] = fcnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int s0 = 0, s1 = 0;
        for (int w = 0; w < (int)(blockDim.x / kWave); ++w) {
            s0 += redc[0][w];
            s1 += redc[1][w];
        }
        a.counts[(long long)item * 2] = s0;
        a.counts[(long long)item * 2 + 1] = s1;
    }
    __syncthreads();   // LDS and the reduction buffers are reused by the next tile
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

// ------------------------------------------------------------- launch templates
// Workgroups of kernel k that fit on the device at once.
template <class K>
hipError_t occupancy(K k, size_t shm, int *max_grid) {
    int per_cu = 0, dev = 0, cus = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kTileWaves * kWave, shm);
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) *max_grid = per_cu * cus;
    return e;
}

template <class Acc, int RA, int RB, int MODE>
hipError_t p1(const Pass1Args<typename AccOps<Acc>::Taps> &a, int grid, hipStream_t s, int *max_grid) {
    const size_t shm = pass1_lds_bytes(a.rows, RB) +
                       ((MODE & kP1Cells) != 0 ? 2 * sizeof(unsigned) * a.cell_rows * a.cell_slots : 0);
    // the map-writing and feature variants always run one tile per workgroup
    if constexpr ((MODE & (kP1Maps | kP1Cells)) != 0) {
        if (max_grid) return occupancy(pass1_kernel<Acc, RA, RB, MODE, false>, shm, max_grid);
        hipLaunchKernelGGL((pass1_kernel<Acc, RA, RB, MODE, false>), dim3(a.L.total1),
                           dim3(kTileWaves * kWave), shm, s, a);
    } else {
        if (max_grid) return occupancy(pass1_kernel<Acc, RA, RB, MODE, true>, shm, max_grid);
        if (grid >= a.L.total1)
            hipLaunchKernelGGL((pass1_kernel<Acc, RA, RB, MODE, false>), dim3(a.L.total1),
                               dim3(kTileWaves * kWave), shm, s, a);
        else
            hipLaunchKernelGGL((pass1_kernel<Acc, RA, RB, MODE, true>), dim3(grid),
                               dim3(kTileWaves * kWave), shm, s, a);
    }
    return hipGetLastError();
}

template <class Acc, int RA, int RB, int MED>
hipError_t p2m(const Pass2Args<typename AccOps<Acc>::Taps> &a, int grid, hipStream_t s, int *max_grid) {
    const size_t shm = lds_bytes(a.rows, kHalo2, RB);
    if constexpr (MED < 0) {   // gated variants run one tile per workgroup
        if (max_grid) return occupancy(pass2_kernel<Acc, RA, RB, MED, false>, shm, max_grid);
        hipLaunchKernelGGL((pass2_kernel<Acc, RA, RB, MED, false>), dim3(a.L.total2),
                           dim3(kTileWaves * kWave), shm, s, a);
    } else {
        if (max_grid) return occupancy(pass2_kernel<Acc, RA, RB, MED, true>, shm, max_grid);
        if (grid >= a.L.total2)
            hipLaunchKernelGGL((pass2_kernel<Acc, RA, RB, MED, false>), dim3(a.L.total2),
                               dim3(kTileWaves * kWave), shm, s, a);
        else
            hipLaunchKernelGGL((pass2_kernel<Acc, RA, RB, MED, true>), dim3(grid),
                               dim3(kTileWaves * kWave), shm, s, a);
    }
    return hipGetLastError();
}
template <class Acc, int RA, int RB>
hipError_t p2(const Pass2Args<typename AccOps<Acc>::Taps> &a, int grid, hipStream_t s, int *max_grid) {
    if (a.med_flags) {   // gated: one workgroup per tile
        const int g = max_grid ? 0 : a.L.total2;
        if (a.median_size == 3) return p2m<Acc, RA, RB, -3>(a, g, s, max_grid);
        return p2m<Acc, RA, RB, -5>(a, g, s, max_grid);
    }
    if (!a.smooth) return p2m<Acc, RA, RB, 0>(a, grid, s, max_grid);
    if (a.median_size == 3) return p2m<Acc, RA, RB, 3>(a, grid, s, max_grid);
    return p2m<Acc, RA, RB, 5>(a, grid, s, max_grid);
}

}  // namespace kern
}  // namespace logfx
