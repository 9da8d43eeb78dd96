// Internal declarations shared by the host runtime and the HIP kernels of
// liblogfx.  Not part of the public ABI (include/logfx.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace logfx {

constexpr int kWave = 64;
constexpr int kTileWaves = 4;                        // waves (column strips) per workgroup
constexpr int kMaxRadius = 4;                        // masks up to 9 x 9
constexpr int kMaxOrbits = (kMaxRadius + 1) * (kMaxRadius + 2) / 2;

// Halo (in L-response pixels) that each pass keeps around its output tile.
//  pass 1: the zero-crossing test needs L at +-1.
//  pass 2: median (+-2) <- local std (+-1) <- zero crossing (+-1) = +-4.
constexpr int kHalo1 = 1;
constexpr int kHalo2 = 4;
//  pass 2 on stored strengths: median (+-2) <- local std (+-1) = +-3;
//  with the 5x5 first deviation stage, median (+-2) <- 5x5 std (+-2) = +-4.
constexpr int kHalo2Z = 3;
constexpr int kHalo2Z5 = 4;

// Pass-1 variants (bits of its MODE).
constexpr int kP1Maps = 1;     // FP64 maps of L and Z (single images, for inspection)
constexpr int kP1Cells = 2;    // the gate's per-cell sums
constexpr int kP1StoreZ = 4;   // the (Z_1, Z_2) pair of every pixel for pass 2
constexpr int kP1Packed = 8;   // integer path: the LoG on packed 16-bit pixel sums

// Side of the cell grid over which pass 1 sums the smoothing gate's
// features (kGateCells x kGateCells cells per image).
constexpr int kGateCellsLog2 = 7;
constexpr int kGateCells = 1 << kGateCellsLog2;

// Orbit index of the D4 orbit {(+-i, +-j), (+-j, +-i)}, 0 <= j <= i.
__host__ __device__ constexpr int orbit_index(int i, int j) { return i * (i + 1) / 2 + j; }

// Packed form of the integer LoG (kP1Packed).  With v(d, c) the sum of
// the pixels at row offsets +-d and column offsets +-c (v(0, 0) the centre,
// v(d, 0) two pixels, v(0, c) two, v(d, c) four), each entry lies in exactly
// one D4 orbit, that of (max(d, c), min(d, c)), so
//   L = sum over d, c in 0..R of k'(d, c) v(d, c),  k'(d, c) = k_orbit.
// Per row offset d the entries are packed in 16-bit halves, kPkPerRow
// words: (v(d, 0), unused), (v(d, 1), v(d, 2)), (v(d, 3), v(d, 4)); the
// taps k' are packed the same way (0 in unused halves and past the mask's
// radius), word d * kPkPerRow + m, and multiplied two at a time
// (v_dot2_i32_i16).  The centre v(0, 0) (one pixel) takes the orbit tap k[0]
// of the 32-bit form in a 24-bit multiply, since that tap alone may exceed
// 16 bits; word 0 is unused.  Valid when every v fits int16 (pixels below
// 2^13) and every other tap does too; the host checks both.
constexpr int kPkPerRow = 3;
constexpr int kPkTaps = (kMaxRadius + 1) * kPkPerRow;

// Orbit taps of both masks, in integer grid units.  The integer path keeps
// them as int (they fit 24-bit signed), and in the packed form above when
// it applies; the FP64 path as double.
struct OrbitTapsI {
    int k[2][kMaxOrbits];
    unsigned pk[2][kPkTaps];
};
struct OrbitTapsD { double k[2][kMaxOrbits]; };

// Device-side statistics written by the finalize kernel (LoG grid units).
struct DevStats {
    double sum[2];     // sum Z_j
    double sumsq[2];   // sum Z_j^2
    double sigma[2];   // unbiased global standard deviation of Z_j
    double thresh[2];  // T_j
    double thr72[2];   // 72 T_j^2 (compared with 9 sum z^2 - (sum z)^2)
    long long zc[2];   // pixels with Z_j != 0
};

struct ImageDesc {
    const void *data;
    long long H, W, pitch;
    int dtype;   // 0 u8, 1 u16
};

// LDS tile geometry of a pass with halo HL and mask radius rb.  The staged
// columns start at an 8-multiple image column (tiles are 8-multiples wide)
// so that interior rows are copied in whole 8-pixel chunks.
__host__ __device__ constexpr int tile_out_width(int halo) { return kTileWaves * (kWave - 2 * halo); }
__host__ __device__ constexpr int tile_lds_offset(int halo, int rb) { return (8 - (halo + rb) % 8) % 8; }
__host__ __device__ constexpr int tile_lds_stride(int halo, int rb) {
    return (tile_out_width(halo) + 2 * halo + 2 * rb + tile_lds_offset(halo, rb) + 7) / 8 * 8;
}
// The staging loads of the passes that read the image copy 8 pixels at a
// time from the tile origin, so their tiles must be 8-multiples wide.
static_assert(tile_out_width(kHalo1) % 8 == 0 && tile_out_width(kHalo2) % 8 == 0,
              "image-reading passes need 8-multiple tile widths");

// One image of a launch: its input, its output and where its tiles sit in
// the launch's tile list.
struct ImageJob {
    ImageDesc img;
    uint8_t *out;          // pass-2 output (pitch out_pitch); unused by pass 1
    long long out_pitch;
    int tiles_x1, tiles_x2;  // tiles across the image in pass 1 / pass 2
    int base1, base2;        // index of the image's first tile among the launch's tiles
    int ntiles1, ntiles2;
    long long zoff;          // first element of the image's strength pairs in the Z map (H*W of them)
};

// The work of one launch: one image (passed inline) or a batch of images
// (a device table), each cut into tiles.  A workgroup may process several
// tiles (persistent launch) or one (grid = number of tiles).
struct Launch {
    int nimg;
    ImageJob one;            // the image when nimg == 1
    const ImageJob *jobs;    // device table of nimg images when nimg > 1
    const int *owner1;       // [total1] image of each pass-1 tile (nimg > 1)
    const int *owner2;       // [total2] image of each pass-2 tile (nimg > 1)
    int total1, total2;      // tiles of all images, pass 1 / pass 2
};

template <class Taps>
struct Pass1Args {
    Launch L;
    Taps taps;
    double zc_thr[2];      // zero-crossing threshold per mask, grid units
    int zc_thr_i[2];       // the same for integer strengths: floor, capped at INT_MAX
    int rows;              // output rows per wave strip
    double *partials;      // [total1][4]: sum Z1, sum Z2, sum Z1^2, sum Z2^2 per tile
    long long *counts;     // [total1][2]: crossings of mask 1, mask 2 per tile
    // Optional FP64 maps of a single image (LoG units = grid units * unit[j]).
    double *dbgL[2];
    double *dbgZ[2];
    double unit[2];
    // Strength pairs (kP1StoreZ): int2 (integer path) or double2 (FP64
    // path) per pixel, image i at element jobs[i].zoff, row pitch W.
    void *zmap;
    // Gate features (kP1Cells): [nimg][2][cells] counters, zeroed before
    // the launch; plane 0 sums pixel values, plane 1 sums
    // [Z_1 != 0] + 2^32 [Z_2 != 0] (every cell must hold < 2^32 pixels).
    // Each image is cut into 2^cells_ly rows by 2^cells_lx columns of cells
    // (kGateCells x kGateCells, or that grid per region when the gate
    // decides per region of a single image).
    unsigned long long *cells;
    int cells_lx, cells_ly;
    // LDS slots of the per-tile cell sums (kP1Cells): cell_rows x cell_slots,
    // at least the cell rows and the cell columns any tile of the launch
    // spans.
    int cell_slots, cell_rows;
};

template <class Taps>
struct Pass2Args {
    Launch L;
    Taps taps;
    double zc_thr[2];
    int zc_thr_i[2];
    int rows;
    const DevStats *stats;  // [nimg] thresholds from the finalize kernel
    int *counts;            // [total2][2]: E pixels, output pixels per tile
    int smooth;             // 0 = E, 1 = hybrid median of E
    int median_size;        // 3 or 5
    const int *med_flags;   // [nimg] or nullptr: when given, image i is smoothed iff med_flags[i] != 0
    const void *zmap;       // strength pairs written by pass 1 (pass 2 on stored strengths)
    int std5;               // the 5x5 first stage: E_j also needs s5 > std5_max (stored strengths only)
    double thr600[2];       // 600 (std5_max / unit_j)^2, compared with 25 sum z^2 - (sum z)^2
    uint8_t *out_map;       // or nullptr: output of image i at out_map + jobs[i].zoff, pitch W
                            // (the first level of a median cascade; stored strengths only)
    int region;             // > 0 (single image, gated): med_flags holds one flag per square
    int reg_gx;             // region of this side, reg_gx regions per region row, row-major
};

// One further level of the hybrid median cascade, on maps of 0/1 bytes,
// with the tiling of the stored-strength pass 2 (halo 3, or 4 with the 5x5
// first stage).
struct LevelArgs {
    Launch L;               // the call's images: output maps, tiling
    int rows;               // rows per strip (pass 2's)
    int median_size;        // 3 or 5
    int from_scratch;       // 1: read the scratch maps, write the outputs; 0: the reverse
    uint8_t *scratch;       // image i at scratch + jobs[i].zoff, pitch W
    const int *med_flags;   // [nimg] or nullptr: images whose flag is 0 are copied unfiltered
    int *counts;            // [total2][2] or nullptr: each tile's output count into counts[2 t + 1]
};

struct FinalizeArgs {
    Launch L;
    const double *partials;
    const long long *counts;
    int std_mode;          // 0 relative, 1 absolute
    double std_k;
    double abs_thr[2];     // absolute threshold per mask in grid units (std_mode 1)
    DevStats *stats;       // [nimg]
};

// Launchers (defined in logfx_dispatch.hip).  They return hipSuccess or the
// launch error.  ra <= rb are the radii of the two masks.  grid = number of
// workgroups (at most the number of tiles; fewer makes the launch
// persistent).  max_grid, when non-null, receives the number of workgroups
// that fit on the device at once and nothing is launched.
// mode: a set of kP1* bits; with kP1Maps or kP1Cells one tile per workgroup.
hipError_t launch_pass1_i(int ra, int rb, const Pass1Args<OrbitTapsI> &a, int mode, int grid,
                          hipStream_t s, int *max_grid = nullptr);
hipError_t launch_pass1_d(int ra, int rb, const Pass1Args<OrbitTapsD> &a, int mode, int grid,
                          hipStream_t s, int *max_grid = nullptr);
hipError_t launch_pass2_i(int ra, int rb, const Pass2Args<OrbitTapsI> &a, int grid, hipStream_t s,
                          int *max_grid = nullptr);
hipError_t launch_pass2_d(int ra, int rb, const Pass2Args<OrbitTapsD> &a, int grid, hipStream_t s,
                          int *max_grid = nullptr);
hipError_t launch_finalize(const FinalizeArgs &a, hipStream_t s);
// Pass 2 on the strengths stored by pass 1 (no LoG, no LDS): tiles of
// tile_out_width(kHalo2Z) columns, or tile_out_width(kHalo2Z5) with the 5x5
// first stage (a.std5).
hipError_t launch_pass2z_i(const Pass2Args<OrbitTapsI> &a, int grid, hipStream_t s, int *max_grid = nullptr);
// One further median level (halo 3 or 4, as the pass 2 of the same call).
hipError_t launch_median_level(const LevelArgs &a, int halo, hipStream_t s);
hipError_t launch_pass2z_d(const Pass2Args<OrbitTapsD> &a, int grid, hipStream_t s, int *max_grid = nullptr);

// Static scratch of logfx_extract_noalloc (one array per device, in
// logfx_dispatch.hip): the per-tile sums and counts of both passes and the
// image's statistics, for at most kNoAllocMaxTiles tiles per pass.
constexpr long long kNoAllocMaxTiles = 65536;
constexpr size_t kNoAllocPartialsOff = 0;                                              // double [T][4]
constexpr size_t kNoAllocCounts1Off = kNoAllocPartialsOff + kNoAllocMaxTiles * 4 * sizeof(double);  // i64 [T][2]
constexpr size_t kNoAllocCounts2Off = kNoAllocCounts1Off + kNoAllocMaxTiles * 2 * sizeof(long long); // i32 [T][2]
constexpr size_t kNoAllocStatsOff = kNoAllocCounts2Off + kNoAllocMaxTiles * 2 * sizeof(int);        // DevStats
constexpr size_t kNoAllocBytes = (kNoAllocStatsOff + sizeof(DevStats) + 255) / 256 * 256;
// Device address of that array on `device` (which must be the current
// device), looked up once per device and kept; the array's host-side name is
// not a device address.
hipError_t noalloc_scratch(int device, void **ptr);

// LDS bytes of one workgroup.
inline size_t lds_bytes(int rows, int halo, int rb) {
    return (size_t)tile_lds_stride(halo, rb) * (rows + 2 * halo + 2 * rb) * sizeof(uint16_t);
}
// Pass 1 holds one spare row after the tile's: its row loop reads each row
// one step ahead, so the last step reads the row after the tile.
inline size_t pass1_lds_bytes(int rows, int rb) {
    return lds_bytes(rows + 1, kHalo1, rb);
}

}  // namespace logfx
