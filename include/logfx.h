/*
 * logfx.h -- C ABI of liblogfx, an MI355X (gfx950) implementation of the
 * feature-extraction pipeline of Tejaswi, Rao, Nair and Prasad, "GPU
 * accelerated automated feature extraction from satellite images"
 * (arXiv:1304.3992):
 *
 *   two Laplacian-of-Gaussian responses (Sec. 3.1, eq. (1); Sec. 4.1),
 *   four-neighbour zero crossings with a strength threshold (Sec. 3.2),
 *   local standard-deviation extraction against a threshold (Sec. 3.3,
 *   eq. (2); Sec. 4.1), OR of the two extracted maps (abstract; Sec. 4.1),
 *   optional hybrid median smoothing (Sec. 3.4; abstract).
 *
 * Conventions shared by every entry point
 *   - Return value: LOGFX_OK (0) or a positive logfx_status.  No call aborts
 *     the process.  On a non-OK return the outputs are undefined and
 *     logfx_last_error() describes the failure.
 *   - Images and outputs are DEVICE pointers owned by the caller (typically
 *     torch tensors).  Mask taps and report structs are HOST memory.
 *   - Work is enqueued on the caller's HIP stream (hipStream_t passed as
 *     void*; NULL = the default stream) and runs asynchronously, except
 *     that passing a non-NULL report makes the call wait for its stream.
 *   - Images are row-major with a pitch in elements (pitch >= width).
 *     Outputs are dense: pitch = width.
 *   - Every stage reads its input through clamp-to-edge indexing (the
 *     padding of Sec. 4.1, whose values the paper does not give).
 *   - A context owns device scratch memory and is used by one host thread
 *     at a time; calls on one context are ordered by the caller's streams.
 */
#ifndef LOGFX_H
#define LOGFX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LOGFX_OK = 0,
    LOGFX_EINVAL = 1,       /* null pointer, bad size, bad enum value */
    LOGFX_EUNSUPPORTED = 2, /* valid request this build cannot run exactly */
    LOGFX_ENOMEM = 3,       /* device scratch allocation failed */
    LOGFX_EDEVICE = 4       /* a HIP call failed (text in logfx_last_error) */
} logfx_status;

enum { LOGFX_U8 = 0, LOGFX_U16 = 1 };
enum { LOGFX_STD_REL = 0, LOGFX_STD_ABS = 1 };
enum { LOGFX_SMOOTH_NEVER = 0, LOGFX_SMOOTH_ALWAYS = 1 };
/* Arithmetic used for the LoG sums (report.path). */
enum { LOGFX_PATH_INT32 = 0, LOGFX_PATH_FP64 = 1 };

typedef struct logfx_ctx logfx_ctx;

/* One image (a panchromatic scene or one band of a multispectral scene,
 * Sec. 4).  data: device pointer; dtype: LOGFX_U8 or LOGFX_U16; bits: number
 * of significant bits (1..8 for U8, 1..16 for U16; 0 = the full width) --
 * every pixel must be < 2^bits, the exactness bound below depends on it. */
typedef struct {
    const void *data;
    int32_t dtype;
    int32_t bits;
    int64_t height, width, pitch;
} logfx_image;

/* A square LoG mask: size x size taps, row-major, HOST memory, copied
 * during the call.  size is odd, 1..9.  The taps must be symmetric under
 * the eight symmetries of the square (as every sampled eq. (1) mask is) and
 * lie on a common power-of-two grid u (taps = k_i * u, k_i integers) with
 * sum|k_i| * (2^bits - 1) < 2^52, so that every LoG sum is exact in any
 * order; otherwise the call returns LOGFX_EUNSUPPORTED.
 * logfx_make_log_mask() builds such masks. */
typedef struct {
    int32_t size;
    const float *taps;
} logfx_mask;

/* Parameters of the pipeline, as the paper states the problem (Sec. 4.1):
 * the two LoG masks, the zero-crossing threshold, the standard-deviation
 * threshold and the smoothing choice.
 *   zc_thresh  : a crossing is kept when its strength (range of the LoG over
 *                the pixel and its four neighbours) exceeds it (Sec. 3.2).
 *                LoG response units, >= 0.
 *   std_mode   : LOGFX_STD_REL: T_j = std_k * (global unbiased standard
 *                deviation of mask j's crossing-strength map);
 *                LOGFX_STD_ABS: T_j = std_k.
 *   std_k      : >= 0.
 *   std5_max   : the paper's 5x5 first stage (Sec. 4.1).  Must be < 0 (off)
 *                in this build; >= 0 returns LOGFX_EUNSUPPORTED.
 *   smooth     : LOGFX_SMOOTH_NEVER or LOGFX_SMOOTH_ALWAYS (hybrid median).
 *   median_size: 3 or 5 (window of the hybrid median, Sec. 3.4).
 *   flags      : reserved, must be 0. */
typedef struct {
    logfx_mask mask[2];
    double zc_thresh;
    int32_t std_mode;
    double std_k;
    double std5_max;
    int32_t smooth;
    int32_t median_size;
    uint32_t flags;
} logfx_params;

/* Filled when a call is given a report (the call then waits for its
 * stream).  sigma_g and thresh are in LoG response units. */
typedef struct {
    int64_t pixels;
    double sigma_g[2];    /* global standard deviation of Z_j (eq. (2))   */
    double thresh[2];     /* T_j                                           */
    int64_t zc_count[2];  /* pixels with Z_j != 0                          */
    int64_t extracted;    /* pixels with E = E_1 OR E_2 set                */
    int64_t output;       /* pixels set in the output (F, or E unsmoothed) */
    int32_t path;         /* LOGFX_PATH_INT32 or LOGFX_PATH_FP64           */
    int32_t smoothed;     /* 1 if the hybrid median was applied            */
} logfx_report;

/* Library version string (static storage). */
const char *logfx_version(void);

/* Create a context on HIP device `device`.  *out receives the context. */
int logfx_create(logfx_ctx **out, int device);

/* Free a context and all its device memory.  NULL is accepted. */
int logfx_destroy(logfx_ctx *ctx);

/* Text of the last error on this context ("" if none).  Valid until the
 * next call on the context.  NULL ctx gives the last error of
 * logfx_create / logfx_make_log_mask on this thread. */
const char *logfx_last_error(const logfx_ctx *ctx);

/* Build a zero-sum LoG mask from eq. (1) (Sec. 3.1): sample it at integer
 * offsets of a size x size window, remove the mean, snap every tap to the
 * grid u = 2^(e + 1 - grid_bits) where 2^e <= max|tap| < 2^(e+1) (round half
 * to even), and subtract the integer sum from the centre tap so the sum is
 * exactly zero.  size: odd 1..15; sigma > 0; grid_bits 2..23.
 * taps_out: HOST, size*size floats.  unit_out (nullable): receives u.
 * Host-only, needs no context or device. */
int logfx_make_log_mask(int32_t size, double sigma, int32_t grid_bits, float *taps_out,
                        double *unit_out);

/* Validate an image descriptor and parameters without touching a device:
 * the same checks logfx_extract makes before it enqueues work (argument
 * ranges, mask symmetry, the exactness bound).  img->data must be non-NULL
 * but is not dereferenced.  path_out (nullable) receives the arithmetic path
 * (LOGFX_PATH_INT32 when sum|k| * (2^bits - 1) < 2^30, else
 * LOGFX_PATH_FP64).  Host-only. */
int logfx_check_params(const logfx_image *img, const logfx_params *p, int32_t *path_out);

/* The whole pipeline on one image (Sec. 4.1, Fig. 1 flow):
 *   L_j = LoG response of mask j; Z_j = crossing strength map of L_j;
 *   E_j = [3x3 local standard deviation of Z_j > T_j]; E = E_1 OR E_2;
 *   out = hybrid_median(E) if p->smooth, else E.
 * out: DEVICE, height*width bytes (0/1), pitch = width, caller-owned.
 * rep: nullable; if given the call waits for `stream` and fills it. */
int logfx_extract(logfx_ctx *ctx, const logfx_image *img, const logfx_params *p, uint8_t *out,
                  logfx_report *rep, void *stream);

/* The first half of the pipeline alone, for inspection and testing: the two
 * LoG responses (Sec. 4.1) and the two crossing-strength maps (Sec. 3.2) as
 * FP64 maps in LoG response units.  Each output is a DEVICE array of
 * height*width doubles (pitch = width) or NULL to skip it.  Same
 * parameters and checks as logfx_extract (only mask, zc_thresh are used). */
int logfx_extract_maps(logfx_ctx *ctx, const logfx_image *img, const logfx_params *p,
                       double *L1, double *L2, double *Z1, double *Z2, void *stream);

/* Many images in one call (a batch of scene tiles of uneven sizes, or the
 * bands of a multispectral scene, Sec. 4.2).  Every image runs the whole
 * pipeline on its own (its own global deviation and thresholds); all share
 * the parameters, dtype and bits.  imgs: HOST array of n descriptors;
 * outs: HOST array of n DEVICE output pointers (height*width bytes each).
 * reps: HOST array of n reports or NULL (given: the call waits).
 * The tiles of all images run in one launch per pass: one workgroup per
 * tile, or, with LOGFX_OPT_PERSISTENT set, a persistent grid of the
 * workgroups that fit on the device walking all tiles; the launches are
 * replayed from a captured hipGraph unless LOGFX_OPT_GRAPH is 0 (the graph
 * is re-captured when the batch geometry or parameters change).  The image table is uploaded from pinned memory on
 * `stream` before the launches. */
int logfx_extract_batch(logfx_ctx *ctx, int32_t n, const logfx_image *imgs, const logfx_params *p,
                        uint8_t *const *outs, logfx_report *reps, void *stream);

/* Context options (logfx_set_option / logfx_get_option). */
enum {
    LOGFX_OPT_ROWS1 = 1,      /* output rows per wave strip in pass 1 (1..1024, default 64) */
    LOGFX_OPT_ROWS2 = 2,      /* the same for pass 2 (default 64) */
    LOGFX_OPT_PERSISTENT = 3, /* batches: 1 = persistent launch, 0 = one workgroup per tile (default) */
    LOGFX_OPT_GRAPH = 4       /* batches: 1 = replay a captured hipGraph (default), 0 = direct launches */
};
int logfx_set_option(logfx_ctx *ctx, int32_t option, int64_t value);
int logfx_get_option(logfx_ctx *ctx, int32_t option, int64_t *value);

/* Autotuner (the launch-parameter sweep of Table 4, Sec. 6.2.3, made
 * automatic).  Runs the given call (one image, or a batch when n > 1) with
 * each candidate strip height for pass 1 and pass 2 (32, 48, 64, 96 rows,
 * as far as they fit in LDS) and, for batches, with and without the
 * persistent launch, `reps` timed repetitions each, and keeps the fastest
 * in the context (LOGFX_OPT_ROWS1/ROWS2/PERSISTENT).  The outputs are
 * written as by the call itself.  cache_path (nullable): a text file of
 * JSON lines keyed by device architecture, arithmetic path, mask radii,
 * pixel type, smoothing and batch/single; an entry found there is applied
 * without measuring, a new result is appended.  res (nullable) receives the
 * choice. */
typedef struct {
    int32_t rows1, rows2, persistent;
    int32_t from_cache;   /* 1 if taken from the cache file */
    double ms;            /* milliseconds of one call with the choice */
} logfx_tune_result;
int logfx_tune(logfx_ctx *ctx, int32_t n, const logfx_image *imgs, const logfx_params *p,
               uint8_t *const *outs, int32_t reps, const char *cache_path, logfx_tune_result *res,
               void *stream);

/* Kernel timing (the split of Table 6 in Sec. 7 between transfers and
 * kernel time, refined per kernel).  While enabled, every extract call on
 * the context records HIP events around its kernels on the call's stream.
 * logfx_timing_read waits for the recorded events and returns summed
 * milliseconds in ms_out[0..3]: pass 1, the finalize kernel, pass 2 (direct
 * launches only; a graph replay is timed as a whole) and the whole call;
 * *calls_out (nullable) receives the number of timed calls.  It starts a new
 * accumulation, as does enabling or disabling. */
int logfx_timing_enable(logfx_ctx *ctx, int on);
int logfx_timing_read(logfx_ctx *ctx, double *ms_out, int64_t *calls_out);

#ifdef __cplusplus
}
#endif

#endif /* LOGFX_H */
