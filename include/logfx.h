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
 *   - Environment: LOGFX_LOG=1 writes one line per call and every error to
 *     stderr; LOGFX_TUNE_CACHE names the autotuner's cache file when
 *     logfx_tune is given none; LOGFX_TILE="rows1,rows2" sets a new
 *     context's strip heights; LOGFX_FAIL_ALLOC=n makes the n-th device
 *     allocation of a new context fail (a test hook).
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
/* Smoothing choice (params.smooth).  GATE: the smoothing gate (a small CNN,
 * see logfx_gate below) decides per image whether the hybrid median is
 * applied; with no gate parameters loaded in the context it falls back to
 * ALWAYS and the report says so. */
enum { LOGFX_SMOOTH_NEVER = 0, LOGFX_SMOOTH_ALWAYS = 1, LOGFX_SMOOTH_GATE = 2 };
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
 *   std5_max   : the paper's 5x5 first stage (Sec. 4.1).  < 0: off.  >= 0
 *                (LoG response units): a pixel of mask j is extracted only
 *                if the unbiased deviation of Z_j over its clamped 5 x 5
 *                window also exceeds std5_max.  Runs on the strengths
 *                stored by pass 1 whatever LOGFX_OPT_STORE_Z says
 *                (LOGFX_ENOMEM if their memory cannot be had).  NaN:
 *                LOGFX_EINVAL.
 *   smooth     : LOGFX_SMOOTH_NEVER, LOGFX_SMOOTH_ALWAYS (hybrid median) or
 *                LOGFX_SMOOTH_GATE (the gate chooses per image).
 *   median_size: 3 or 5 (window of the hybrid median, Sec. 3.4).
 *   flags      : 0, or LOGFX_ALLOW_INEXACT: a mask pair whose taps cannot
 *                be summed exactly in FP64 (LOGFX_EUNSUPPORTED without the
 *                flag) runs on the FP64 path with rounded sums, and the
 *                report says so (inexact = 1).  Other bits: LOGFX_EINVAL.
 *   median_cascade: further levels of the hybrid median (Sec. 3.4: the
 *                filter may be applied repeatedly; Sec. 4.2: the map passes
 *                through levels of larger and smaller windows).  Entry i,
 *                3 or 5, is the window of level i + 2, applied to the
 *                output of level i + 1; a 0 ends the list (all 0: one
 *                level).  The levels apply wherever the first one does
 *                (LOGFX_SMOOTH_ALWAYS, or LOGFX_SMOOTH_GATE on the images
 *                the gate smooths).  Calls with further levels store the
 *                strengths between the passes whatever LOGFX_OPT_STORE_Z
 *                says and keep a 1-byte-per-pixel map in the context.
 *   gate_region: 0, or the side R of the square regions in which the gate
 *                decides the median of a single image (seamless scene
 *                mode: a scene cut into tiles only for the smoothing
 *                choice, which Sec. 1 makes per image).  The image keeps one
 *                global deviation and threshold per mask and reads its
 *                neighbours across region borders; each region gets the
 *                gate's features of its own 128 x 128 cells and its own
 *                decision, and its pixels are F where the region is
 *                smoothed, E elsewhere.  Needs smooth = LOGFX_SMOOTH_GATE,
 *                128 <= R < 2^23, height and width multiples of R, a
 *                power-of-two number of regions across and down (at most
 *                LOGFX_GATE_MAX_BATCH in all), no median_cascade, and a
 *                single-image call (LOGFX_EINVAL otherwise).  Stores the
 *                strengths between the passes whatever LOGFX_OPT_STORE_Z
 *                says.  Without gate parameters the call falls back to
 *                LOGFX_SMOOTH_ALWAYS, as GATE does. */
#define LOGFX_ALLOW_INEXACT 1u

typedef struct {
    logfx_mask mask[2];
    double zc_thresh;
    int32_t std_mode;
    double std_k;
    double std5_max;
    int32_t smooth;
    int32_t median_size;
    uint32_t flags;
    int32_t median_cascade[3];
    int32_t gate_region;
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
    int32_t gated;        /* 1 if the gate took the smoothing decision     */
    int32_t gate_fallback;/* 1 if GATE was asked with no gate parameters   */
    double gate_logit;    /* the gate's logit (gated calls), else 0        */
    int32_t inexact;      /* 1 if the LoG sums were rounded (LOGFX_ALLOW_INEXACT) */
    int32_t regions;      /* gate_region calls: number of regions, else 0  */
    int32_t regions_smoothed; /* of them, the regions the gate smoothed   */
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

/* logfx_extract for callers that cannot allocate memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation.
 * The same pipeline and the same output bytes as logfx_extract; the call
 * allocates nothing, host or device.  Its scratch (per-tile sums and counts
 * of both passes, the image's statistics) is a fixed static array of 3.5
 * MiB on each device, held until the process ends; pass 2 recomputes the
 * crossing strengths (as LOGFX_OPT_STORE_Z = 0 does) instead of storing
 * them.  The tile heights come from ctx's options; no report, no timing.
 * Limits (LOGFX_EINVAL beyond them, before anything is enqueued): at most
 * 65536 tiles per pass -- with the default 64-row strips about 0.94
 * Gpixel, e.g. 30000 x 30000 -- and no std5_max >= 0, median_cascade,
 * gate_region, nor LOGFX_SMOOTH_GATE with gate parameters loaded (GATE
 * without parameters runs as ALWAYS).  Every call on a device shares that
 * device's array: calls that overlap in time on one device (other streams,
 * other contexts, other threads) race and give undefined output; calls
 * ordered on one stream are safe.  Other behaviour as logfx_extract. */
int logfx_extract_noalloc(logfx_ctx *ctx, const logfx_image *img, const logfx_params *p, uint8_t *out,
                          void *stream);

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
 * `stream` before the launches.
 * With p->smooth = LOGFX_SMOOTH_GATE (and gate parameters in the context)
 * pass 1 also sums each image's gate features, the network decides between
 * pass 1 and pass 2 which images get the hybrid median, and each report's
 * smoothed / gated / gate_logit give the decision (at most
 * LOGFX_GATE_MAX_BATCH images per call; every gate cell must hold fewer than
 * 2^32 pixels). */
int logfx_extract_batch(logfx_ctx *ctx, int32_t n, const logfx_image *imgs, const logfx_params *p,
                        uint8_t *const *outs, logfx_report *reps, void *stream);

/* Context options (logfx_set_option / logfx_get_option). */
enum {
    LOGFX_OPT_ROWS1 = 1,      /* output rows per wave strip in pass 1 (1..1024, default 64) */
    LOGFX_OPT_ROWS2 = 2,      /* the same for pass 2 (default 64) */
    LOGFX_OPT_PERSISTENT = 3, /* batches: 1 = persistent launch, 0 = one workgroup per tile (default) */
    LOGFX_OPT_GRAPH = 4,      /* batches: 1 = replay a captured hipGraph (default), 0 = direct launches */
    LOGFX_OPT_STORE_Z = 5,    /* 1 (default) = pass 1 stores the crossing strengths of every pixel in
                                 context memory (8 bytes per pixel on the integer path, 16 on FP64) and
                                 pass 2 reads them; 0 = pass 2 recomputes them from the image (no such
                                 memory).  Both give the same output; a call whose strength memory
                                 cannot be allocated recomputes. */
    LOGFX_OPT_PACKED_LOG = 6  /* 1 (default) = on the integer path, pass 1 evaluates the LoG on packed
                                 16-bit sums of pixel pairs (two taps per multiply-add) where the
                                 pixels have at most 13 bits and every tap but the centre fits 16
                                 bits; 0 = always the 32-bit form.  Both give the same bits. */
};
int logfx_set_option(logfx_ctx *ctx, int32_t option, int64_t value);
int logfx_get_option(logfx_ctx *ctx, int32_t option, int64_t *value);

/* Autotuner (the launch-parameter sweep of Table 4, Sec. 6.2.3, made
 * automatic).  Runs the given call (one image, or a batch when n > 1) with
 * each candidate strip height for pass 1 and pass 2 (32, 40, 48, 56, 64, 96
 * rows, as far as they fit in LDS) and, for batches, with and without the
 * persistent launch, `reps` timed repetitions each, in two round-robin
 * rounds (each candidate keeps its faster round), and keeps the fastest in
 * the context (LOGFX_OPT_ROWS1/ROWS2/PERSISTENT).  The outputs are
 * written as by the call itself.  cache_path (nullable): a text file of
 * JSON lines keyed by device architecture, arithmetic path, mask radii,
 * pixel type, smoothing and batch/single; an entry found there is applied
 * without measuring, a new result is appended.  res (nullable) receives the
 * choice.  cache_path NULL: the file LOGFX_TUNE_CACHE names, if set. */
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
 * milliseconds in ms_out[0..3]: pass 1, the finalize kernel (with the
 * gate's features and network when it decides), pass 2 (direct launches
 * only; a graph replay is timed as a whole) and the whole call;
 * *calls_out (nullable) receives the number of timed calls.  It starts a new
 * accumulation, as does enabling or disabling. */
int logfx_timing_enable(logfx_ctx *ctx, int on);
int logfx_timing_read(logfx_ctx *ctx, double *ms_out, int64_t *calls_out);

/* ------------------------------------------------------------------------
 * The smoothing gate.  The paper leaves the choice to smooth the extracted
 * map or not to the user, according to its noise (abstract; Sec. 4).  The
 * gate takes it per image from features that pass 1 gathers on the way:
 *
 *   features  3 x 128 x 128 per image.  The image is cut into 128 x 128
 *             cells (row y and column x fall in cell (floor(128 y / H),
 *             floor(128 x / W)); cells of images smaller than 128 in a
 *             direction may be empty and give 0).  Per cell: the mean pixel
 *             value / (2^bits - 1), and the fractions of pixels with a
 *             non-zero crossing strength Z_1, Z_2 (Sec. 3.2).  Computed in
 *             FP64 from exact integer sums, stored as bfloat16 (round to
 *             nearest even), [n][3][128][128], channel order as listed.
 *   network   conv 3x3, stride 2, zero padding 1, 3 -> 16 channels, ReLU;
 *             conv 16 -> 32, ReLU; conv 32 -> 32, ReLU (128 -> 64 -> 32 ->
 *             16); mean over the 16 x 16 positions; linear 32 -> 1 logit.
 *             Smooth iff logit > 0.
 *   numbers   bfloat16 features, convolution weights and stored
 *             activations (and their masked gradients); FP32 accumulation
 *             on the matrix cores; FP32 biases, head, loss and optimiser.
 *   training  mean binary cross-entropy with logits; AdamW (beta1 0.9,
 *             beta2 0.999, eps 1e-8, decoupled weight decay 1e-4 on every
 *             parameter) on FP32 master parameters kept in the context.
 *
 * Parameters are a flat FP32 vector of LOGFX_GATE_NPARAM values:
 *   w1[16][3][3][3] b1[16] w2[32][16][3][3] b2[32] w3[32][32][3][3] b3[32]
 *   wf[32] bf[1]   (weights [out][in][ky][kx]; ky, kx = 0..2 for offsets
 *   -1..1).
 * Feature sets for the training calls are DEVICE arrays of bfloat16 bits
 * [N][3][128][128]; idx (DEVICE int32 [B], nullable) selects the B samples
 * of a batch (NULL: samples 0..B-1); labels are DEVICE floats [N] (0 or 1)
 * indexed like the features.  All gate calls are asynchronous on `stream`
 * except the parameter transfers, which complete before they return.
 * ---------------------------------------------------------------------- */
#define LOGFX_GATE_NPARAM 14369
#define LOGFX_GATE_CELLS 128
#define LOGFX_GATE_MAX_BATCH 4096

/* Features of n images (pass 1 of the pipeline with the cell sums; the
 * parameters are those of logfx_extract_batch, smooth is ignored).  Every
 * cell must hold fewer than 2^32 pixels.  feats: DEVICE, n*3*128*128
 * bfloat16 values.  With p->gate_region > 0 (n = 1, smooth =
 * LOGFX_SMOOTH_GATE): one feature set per region, regions row-major, so
 * regions*3*128*128 values. */
int logfx_gate_features(logfx_ctx *ctx, int32_t n, const logfx_image *imgs, const logfx_params *p,
                        uint16_t *feats, void *stream);

/* Set the gate's parameters from HOST memory (n must be LOGFX_GATE_NPARAM)
 * and reset the optimiser state (moments and step count). */
int logfx_gate_set_params(logfx_ctx *ctx, const float *theta, int64_t n);
/* Copy the parameters to HOST memory (waits for the device). */
int logfx_gate_get_params(logfx_ctx *ctx, float *theta, int64_t n);
/* Parameters from / to a file: the 8 bytes "LOGFXGT1", int32 parameter
 * count, int32 0, then the FP32 values, all little-endian.  logfx_gate_load
 * also takes a training-state file (below) and uses its parameters; like
 * logfx_gate_set_params it resets the optimiser state.  A missing, short or
 * corrupt file gives LOGFX_EINVAL and leaves the context's gate as it was
 * (a context without parameters then runs LOGFX_SMOOTH_GATE as ALWAYS and
 * reports gate_fallback). */
int logfx_gate_load(logfx_ctx *ctx, const char *path);
int logfx_gate_save(logfx_ctx *ctx, const char *path);

/* Training state to / from a file, so that training can stop and resume
 * with the same result as an uninterrupted run: the 8 bytes "LOGFXGS1",
 * int32 parameter count, int32 version 1, int64 AdamW step count, then
 * LOGFX_GATE_NPARAM FP32 parameters, first moments and second moments,
 * then a uint64 FNV-1a (64-bit) checksum of every byte before it; all
 * little-endian.  Saving waits for the device and needs parameters in the
 * context.  Loading checks the size, header, checksum and values (finite,
 * second moments >= 0) before it changes anything: LOGFX_EINVAL on any
 * failure, with the context's gate left as it was. */
int logfx_gate_save_state(logfx_ctx *ctx, const char *path);
int logfx_gate_load_state(logfx_ctx *ctx, const char *path);

/* Logits of B samples (1 <= B <= LOGFX_GATE_MAX_BATCH).  logits: DEVICE
 * float[B]. */
int logfx_gate_forward(logfx_ctx *ctx, int32_t B, const uint16_t *feats, const int32_t *idx,
                       float *logits, void *stream);
/* Gradient of the mean loss over B samples with respect to the parameters
 * (forward and backward pass).  grad: DEVICE float[LOGFX_GATE_NPARAM] or
 * NULL (then the context's gradient buffer, which logfx_gate_step uses);
 * loss: DEVICE float[1] or NULL. */
int logfx_gate_backward(logfx_ctx *ctx, int32_t B, const uint16_t *feats, const int32_t *idx,
                        const float *labels, float *grad, float *loss, void *stream);
/* One AdamW step with learning rate lr on a gradient (DEVICE, or NULL for
 * the context's gradient buffer). */
int logfx_gate_step(logfx_ctx *ctx, const float *grad, double lr, void *stream);

/* The gate on n images: features, network, decision.  logits: DEVICE
 * float[n] or NULL; decisions: DEVICE uint8[n] (1 = smooth) or NULL.
 * Needs gate parameters (LOGFX_EINVAL otherwise).  With p->gate_region > 0
 * (n = 1): one logit and decision per region, regions row-major: the
 * decisions logfx_extract takes with the same parameters. */
int logfx_gate(logfx_ctx *ctx, int32_t n, const logfx_image *imgs, const logfx_params *p, float *logits,
               uint8_t *decisions, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* LOGFX_H */
