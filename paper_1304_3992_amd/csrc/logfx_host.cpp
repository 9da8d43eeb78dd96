// Host runtime and C ABI of liblogfx (declared in include/logfx.h).
//
// Validates arguments and masks, picks the exact arithmetic path, owns the
// per-context device scratch (per-tile partial sums, counters, the global
// statistics) and enqueues   pass 1 -> finalize -> pass 2   on the caller's
// stream.  No compute happens on the host.
#include "logfx.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "logfx_internal.h"

using namespace logfx;

namespace {

thread_local std::string g_thread_error;

// Output rows per wave strip of each pass (tiles are kTileWaves strips wide).
struct TileCfg {
    int rows1 = 64;  // pass 1
    int rows2 = 64;  // pass 2
};

// LOGFX_TILE="rows1,rows2" overrides the defaults (used by the tuner and
// the tests).
TileCfg tile_cfg_from_env() {
    TileCfg t;
    if (const char *s = std::getenv("LOGFX_TILE")) {
        int a, b;
        if (std::sscanf(s, "%d,%d", &a, &b) == 2 && a >= 1 && a <= 1024 && b >= 1 && b <= 1024)
            t.rows1 = a, t.rows2 = b;
    }
    return t;
}

}  // namespace

struct logfx_ctx {
    int device = 0;
    std::string err;
    TileCfg tiles;
    // device scratch
    double *partials = nullptr;      // [cap1][4]
    long long *counts1 = nullptr;    // [cap1][2]
    int *counts2 = nullptr;          // [cap2][2]
    DevStats *stats = nullptr;
    long long cap1 = 0, cap2 = 0;
    // pinned host mirror for reports
    DevStats *h_stats = nullptr;
    int *h_counts2 = nullptr;
    long long h_cap2 = 0;
    // kernel timing: 4 events per timed call (start, after pass 1, after
    // finalize, after pass 2), reused across accumulations
    bool timing = false;
    std::vector<hipEvent_t> events;
    long long timed_calls = 0;
    int alloc_count = 0;
    int fail_alloc_at = -1;          // test hook: LOGFX_FAIL_ALLOC=n fails the n-th allocation
};

namespace {

int set_err(logfx_ctx *ctx, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    else g_thread_error = buf;
    return code;
}

int hip_err(logfx_ctx *ctx, hipError_t e, const char *what) {
    return set_err(ctx, e == hipErrorOutOfMemory ? LOGFX_ENOMEM : LOGFX_EDEVICE, "%s: %s", what,
                   hipGetErrorString(e));
}

struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        int cur;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

template <class T>
int dev_alloc(logfx_ctx *ctx, T **p, size_t count) {
    ++ctx->alloc_count;
    if (ctx->fail_alloc_at > 0 && ctx->alloc_count == ctx->fail_alloc_at)
        return set_err(ctx, LOGFX_ENOMEM, "device allocation %d failed (LOGFX_FAIL_ALLOC)",
                       ctx->alloc_count);
    hipError_t e = hipMalloc((void **)p, count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return hip_err(ctx, e, "hipMalloc");
    }
    return LOGFX_OK;
}

int ensure_scratch(logfx_ctx *ctx, long long n1, long long n2) {
    int rc;
    if (!ctx->stats && (rc = dev_alloc(ctx, &ctx->stats, 1)) != LOGFX_OK) return rc;
    if (n1 > ctx->cap1) {
        (void)hipFree(ctx->partials);
        (void)hipFree(ctx->counts1);
        ctx->partials = nullptr, ctx->counts1 = nullptr, ctx->cap1 = 0;
        if ((rc = dev_alloc(ctx, &ctx->partials, (size_t)n1 * 4)) != LOGFX_OK) return rc;
        if ((rc = dev_alloc(ctx, &ctx->counts1, (size_t)n1 * 2)) != LOGFX_OK) return rc;
        ctx->cap1 = n1;
    }
    if (n2 > ctx->cap2) {
        (void)hipFree(ctx->counts2);
        ctx->counts2 = nullptr, ctx->cap2 = 0;
        if ((rc = dev_alloc(ctx, &ctx->counts2, (size_t)n2 * 2)) != LOGFX_OK) return rc;
        ctx->cap2 = n2;
    }
    return LOGFX_OK;
}

int ensure_host(logfx_ctx *ctx, long long n2) {
    if (!ctx->h_stats) {
        hipError_t e = hipHostMalloc((void **)&ctx->h_stats, sizeof(DevStats), hipHostMallocDefault);
        if (e != hipSuccess) return hip_err(ctx, e, "hipHostMalloc");
    }
    if (n2 > ctx->h_cap2) {
        if (ctx->h_counts2) (void)hipHostFree(ctx->h_counts2);
        ctx->h_counts2 = nullptr, ctx->h_cap2 = 0;
        hipError_t e = hipHostMalloc((void **)&ctx->h_counts2, (size_t)n2 * 2 * sizeof(int),
                                     hipHostMallocDefault);
        if (e != hipSuccess) return hip_err(ctx, e, "hipHostMalloc");
        ctx->h_cap2 = n2;
    }
    return LOGFX_OK;
}

// Events of timed call number `call` (created on first use).
int timing_events(logfx_ctx *ctx, long long call, hipEvent_t *ev) {
    while ((long long)ctx->events.size() < 4 * (call + 1)) {
        hipEvent_t e;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return hip_err(ctx, r, "hipEventCreate");
        ctx->events.push_back(e);
    }
    for (int i = 0; i < 4; ++i) ev[i] = ctx->events[4 * call + i];
    return LOGFX_OK;
}

// ------------------------------------------------------------ mask analysis
struct MaskInfo {
    int size = 0, radius = 0;
    double unit = 1.0;       // grid unit u: taps = k * u
    double k[81];            // integer taps (exact in double)
    double sumabs = 0.0;     // sum |k|
    double maxabs = 0.0;     // max |k|
};

int analyze_mask(logfx_ctx *ctx, const logfx_mask &m, int which, MaskInfo &mi) {
    if (!m.taps) return set_err(ctx, LOGFX_EINVAL, "mask %d: taps is NULL", which);
    if (m.size < 1 || m.size % 2 == 0 || m.size > 15)
        return set_err(ctx, LOGFX_EINVAL, "mask %d: size %d is not odd in 1..15", which, m.size);
    if (m.size > 2 * kMaxRadius + 1)
        return set_err(ctx, LOGFX_EUNSUPPORTED, "mask %d: size %d > 9 is not supported", which,
                       m.size);
    const int s = m.size, r = s / 2;
    mi.size = s;
    mi.radius = r;
    int min_lsb = 1 << 30;
    bool any = false;
    for (int i = 0; i < s * s; ++i) {
        const float t = m.taps[i];
        if (!std::isfinite(t)) return set_err(ctx, LOGFX_EINVAL, "mask %d: tap %d not finite", which, i);
        if (t == 0.0f) continue;
        any = true;
        int e;
        const double fr = std::frexp((double)t, &e);          // |fr| in [0.5, 1)
        long long M = (long long)std::ldexp(std::fabs(fr), 24);  // 24-bit integer mantissa
        int b = 0;
        while (!(M & 1)) M >>= 1, ++b;
        const int lsb = e - 24 + b;
        if (lsb < min_lsb) min_lsb = lsb;
    }
    mi.unit = any ? std::ldexp(1.0, min_lsb) : 1.0;
    mi.sumabs = mi.maxabs = 0.0;
    for (int i = 0; i < s * s; ++i) {
        const double k = (double)m.taps[i] / mi.unit;
        if (std::fabs(k) > 9007199254740992.0)
            return set_err(ctx, LOGFX_EUNSUPPORTED,
                           "mask %d: taps span too many binary orders for exact sums", which);
        mi.k[i] = k;
        mi.sumabs += std::fabs(k);
        if (std::fabs(k) > mi.maxabs) mi.maxabs = std::fabs(k);
    }
    // the eight symmetries of the square grid
    for (int y = 0; y < s; ++y)
        for (int x = 0; x < s; ++x) {
            const float v = m.taps[y * s + x];
            const int ys[4] = {y, s - 1 - y, x, s - 1 - x};
            const int xs[4] = {s - 1 - x, x, y, y};
            for (int q = 0; q < 4; ++q)
                if (m.taps[ys[q] * s + xs[q]] != v)
                    return set_err(ctx, LOGFX_EUNSUPPORTED,
                                   "mask %d is not symmetric under the square's symmetries "
                                   "(asymmetric masks are not supported)", which);
        }
    return LOGFX_OK;
}

struct Plan {
    MaskInfo mi[2];
    int order[2];         // kernel mask slot -> user mask index
    int ra = 1, rb = 1;   // kernel radii, ra <= rb
    int path = LOGFX_PATH_INT32;
    double maxpix = 255.0;
};

int check_all(logfx_ctx *ctx, const logfx_image *img, const logfx_params *p, Plan &pl) {
    if (!img || !p) return set_err(ctx, LOGFX_EINVAL, "image or params is NULL");
    if (!img->data) return set_err(ctx, LOGFX_EINVAL, "image data is NULL");
    if (img->dtype != LOGFX_U8 && img->dtype != LOGFX_U16)
        return set_err(ctx, LOGFX_EINVAL, "unknown dtype %d", img->dtype);
    if (img->height < 1 || img->width < 1)
        return set_err(ctx, LOGFX_EINVAL, "image is empty (%lld x %lld)", (long long)img->height,
                       (long long)img->width);
    if (img->pitch < img->width)
        return set_err(ctx, LOGFX_EINVAL, "pitch %lld < width %lld", (long long)img->pitch,
                       (long long)img->width);
    const int full = img->dtype == LOGFX_U8 ? 8 : 16;
    const int bits = img->bits == 0 ? full : img->bits;
    if (bits < 1 || bits > full) return set_err(ctx, LOGFX_EINVAL, "bits %d not in 1..%d", bits, full);
    if (!(p->zc_thresh >= 0.0) || !std::isfinite(p->zc_thresh))
        return set_err(ctx, LOGFX_EINVAL, "zc_thresh must be finite and >= 0");
    if (p->std_mode != LOGFX_STD_REL && p->std_mode != LOGFX_STD_ABS)
        return set_err(ctx, LOGFX_EINVAL, "unknown std_mode %d", p->std_mode);
    if (!(p->std_k >= 0.0) || !std::isfinite(p->std_k))
        return set_err(ctx, LOGFX_EINVAL, "std_k must be finite and >= 0");
    if (std::isnan(p->std5_max)) return set_err(ctx, LOGFX_EINVAL, "std5_max is NaN");
    if (p->std5_max >= 0.0)
        return set_err(ctx, LOGFX_EUNSUPPORTED, "the 5x5 first deviation stage (std5_max >= 0) "
                                                "is not supported in this build");
    if (p->smooth != LOGFX_SMOOTH_NEVER && p->smooth != LOGFX_SMOOTH_ALWAYS)
        return set_err(ctx, LOGFX_EINVAL, "unknown smooth mode %d", p->smooth);
    if (p->median_size != 3 && p->median_size != 5)
        return set_err(ctx, LOGFX_EINVAL, "median_size %d is not 3 or 5", p->median_size);
    if (p->flags != 0) return set_err(ctx, LOGFX_EINVAL, "flags must be 0");
    int rc;
    for (int j = 0; j < 2; ++j)
        if ((rc = analyze_mask(ctx, p->mask[j], j, pl.mi[j])) != LOGFX_OK) return rc;
    pl.maxpix = std::ldexp(1.0, bits) - 1.0;
    bool int_ok = true, f64_ok = true;
    for (int j = 0; j < 2; ++j) {
        const double bound = pl.mi[j].sumabs * pl.maxpix;
        if (!(bound < 1073741824.0 && pl.mi[j].maxabs < 8388608.0)) int_ok = false;  // 2^30, 2^23
        if (!(bound < 4503599627370496.0)) f64_ok = false;                              // 2^52
    }
    if (!f64_ok)
        return set_err(ctx, LOGFX_EUNSUPPORTED,
                       "mask taps are not exactly summable for %d-bit pixels "
                       "(sum|k| * (2^bits - 1) must stay below 2^52)", bits);
    pl.path = int_ok ? LOGFX_PATH_INT32 : LOGFX_PATH_FP64;
    const int r0 = pl.mi[0].radius, r1 = pl.mi[1].radius;
    if (r0 <= r1) pl.order[0] = 0, pl.order[1] = 1;
    else pl.order[0] = 1, pl.order[1] = 0;
    pl.ra = std::max(1, std::min(r0, r1));
    pl.rb = std::max(1, std::max(r0, r1));
    return LOGFX_OK;
}

template <class Taps, class V>
void fill_taps(const Plan &pl, Taps &t) {
    std::memset(&t, 0, sizeof t);
    for (int slot = 0; slot < 2; ++slot) {
        const MaskInfo &mi = pl.mi[pl.order[slot]];
        const int s = mi.size, r = mi.radius;
        for (int i = 0; i <= r; ++i)
            for (int j = 0; j <= i; ++j) t.k[slot][orbit_index(i, j)] = (V)mi.k[(r + i) * s + (r + j)];
    }
}

struct Geometry {
    int tiles_x1, ntiles1, tiles_x2, ntiles2;
};

int geometry(logfx_ctx *ctx, const logfx_image *img, const Plan &pl, Geometry &g) {
    const TileCfg &t = ctx->tiles;
    const long long H = img->height, W = img->width;
    if (H >= (1LL << 30) || W >= (1LL << 30))
        return set_err(ctx, LOGFX_EUNSUPPORTED, "image sides must be below 2^30");
    const long long tw1 = (long long)kTileWaves * (kWave - 2 * kHalo1);
    const long long tw2 = (long long)kTileWaves * (kWave - 2 * kHalo2);
    const long long tx1 = (W + tw1 - 1) / tw1, ty1 = (H + t.rows1 - 1) / t.rows1;
    const long long tx2 = (W + tw2 - 1) / tw2, ty2 = (H + t.rows2 - 1) / t.rows2;
    if (tx1 * ty1 > 0x7fffffffLL || tx2 * ty2 > 0x7fffffffLL)
        return set_err(ctx, LOGFX_EUNSUPPORTED, "image too large for one launch");
    if (lds_bytes(t.rows1, kHalo1, pl.rb) > 65536 || lds_bytes(t.rows2, kHalo2, pl.rb) > 65536)
        return set_err(ctx, LOGFX_EUNSUPPORTED, "tile configuration exceeds 64 KiB of LDS");
    g.tiles_x1 = (int)tx1, g.ntiles1 = (int)(tx1 * ty1);
    g.tiles_x2 = (int)tx2, g.ntiles2 = (int)(tx2 * ty2);
    return LOGFX_OK;
}

// For an integer strength c and a threshold thr >= 0: c > thr <=> c > floor(thr).
int int_threshold(double thr) {
    const double f = std::floor(thr);
    return f >= 2147483647.0 ? 2147483647 : (int)f;
}

ImageDesc image_desc(const logfx_image *img) {
    ImageDesc d;
    d.data = img->data;
    d.H = img->height;
    d.W = img->width;
    d.pitch = img->pitch;
    d.dtype = img->dtype;
    // 8 pixels per load need the row starts 8-pixel aligned in bytes
    const size_t esz = img->dtype == LOGFX_U16 ? 2 : 1;
    d.vec = ((uintptr_t)img->data % (8 * esz) == 0) && (img->pitch % 8 == 0);
    return d;
}

template <class Taps, class V>
hipError_t launch_p1(const Plan &pl, const Geometry &g, logfx_ctx *ctx, const logfx_image *img,
                     const logfx_params *p, double *const L[2], double *const Z[2], hipStream_t s) {
    Pass1Args<Taps> a;
    std::memset(&a, 0, sizeof a);
    a.img = image_desc(img);
    fill_taps<Taps, V>(pl, a.taps);
    bool dbg = false;
    for (int slot = 0; slot < 2; ++slot) {
        const int u = pl.order[slot];
        a.zc_thr[slot] = p->zc_thresh / pl.mi[u].unit;
        a.zc_thr_i[slot] = int_threshold(a.zc_thr[slot]);
        a.unit[slot] = pl.mi[u].unit;
        a.dbgL[slot] = L ? L[u] : nullptr;
        a.dbgZ[slot] = Z ? Z[u] : nullptr;
        dbg = dbg || a.dbgL[slot] || a.dbgZ[slot];
    }
    a.rows = ctx->tiles.rows1;
    a.tiles_x = g.tiles_x1;
    a.ntiles = g.ntiles1;
    a.partials = ctx->partials;
    a.counts = ctx->counts1;
    if constexpr (sizeof(V) == sizeof(int)) return launch_pass1_i(pl.ra, pl.rb, a, dbg, s);
    else return launch_pass1_d(pl.ra, pl.rb, a, dbg, s);
}

template <class Taps, class V>
hipError_t launch_p2(const Plan &pl, const Geometry &g, logfx_ctx *ctx, const logfx_image *img,
                     const logfx_params *p, uint8_t *out, hipStream_t s) {
    Pass2Args<Taps> a;
    std::memset(&a, 0, sizeof a);
    a.img = image_desc(img);
    fill_taps<Taps, V>(pl, a.taps);
    for (int slot = 0; slot < 2; ++slot) {
        a.zc_thr[slot] = p->zc_thresh / pl.mi[pl.order[slot]].unit;
        a.zc_thr_i[slot] = int_threshold(a.zc_thr[slot]);
    }
    a.rows = ctx->tiles.rows2;
    a.tiles_x = g.tiles_x2;
    a.ntiles = g.ntiles2;
    a.stats = ctx->stats;
    a.out = out;
    a.out_pitch = img->width;
    a.smooth = p->smooth == LOGFX_SMOOTH_ALWAYS;
    a.median_size = p->median_size;
    a.counts = ctx->counts2;
    if constexpr (sizeof(V) == sizeof(int)) return launch_pass2_i(pl.ra, pl.rb, a, s);
    else return launch_pass2_d(pl.ra, pl.rb, a, s);
}

}  // namespace

// ===================================================================== ABI
extern "C" {

const char *logfx_version(void) { return "liblogfx 0.1 (gfx950)"; }

const char *logfx_last_error(const logfx_ctx *ctx) {
    return ctx ? ctx->err.c_str() : g_thread_error.c_str();
}

int logfx_create(logfx_ctx **out, int device) {
    if (!out) return set_err(nullptr, LOGFX_EINVAL, "out is NULL");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n == 0)
        return set_err(nullptr, LOGFX_EDEVICE, "no HIP device available (%s)",
                       e == hipSuccess ? "0 devices" : hipGetErrorString(e));
    if (device < 0 || device >= n)
        return set_err(nullptr, LOGFX_EINVAL, "device %d not in 0..%d", device, n - 1);
    logfx_ctx *ctx = new (std::nothrow) logfx_ctx;
    if (!ctx) return set_err(nullptr, LOGFX_ENOMEM, "out of host memory");
    ctx->device = device;
    ctx->tiles = tile_cfg_from_env();
    if (const char *f = std::getenv("LOGFX_FAIL_ALLOC")) ctx->fail_alloc_at = std::atoi(f);
    *out = ctx;
    return LOGFX_OK;
}

int logfx_destroy(logfx_ctx *ctx) {
    if (!ctx) return LOGFX_OK;
    {
        DeviceGuard g(ctx->device);
        (void)hipFree(ctx->partials);
        (void)hipFree(ctx->counts1);
        (void)hipFree(ctx->counts2);
        (void)hipFree(ctx->stats);
        if (ctx->h_stats) (void)hipHostFree(ctx->h_stats);
        if (ctx->h_counts2) (void)hipHostFree(ctx->h_counts2);
        for (hipEvent_t ev : ctx->events) (void)hipEventDestroy(ev);
    }
    delete ctx;
    return LOGFX_OK;
}

int logfx_make_log_mask(int32_t size, double sigma, int32_t grid_bits, float *taps_out,
                        double *unit_out) {
    if (!taps_out) return set_err(nullptr, LOGFX_EINVAL, "taps_out is NULL");
    if (size < 1 || size % 2 == 0 || size > 15)
        return set_err(nullptr, LOGFX_EINVAL, "size %d is not odd in 1..15", size);
    if (!(sigma > 0.0) || !std::isfinite(sigma))
        return set_err(nullptr, LOGFX_EINVAL, "sigma must be finite and > 0");
    if (grid_bits < 2 || grid_bits > 23)
        return set_err(nullptr, LOGFX_EINVAL, "grid_bits %d not in 2..23", grid_bits);
    const int r = size / 2, n = size * size;
    double v[225];
    double total = 0.0;
    // eq. (1) sampled at integer offsets
    for (int y = -r; y <= r; ++y)
        for (int x = -r; x <= r; ++x) {
            const double q = (double)(x * x + y * y) / (2.0 * sigma * sigma);
            const double val = -1.0 / (M_PI * sigma * sigma * sigma * sigma) * (1.0 - q) * std::exp(-q);
            v[(y + r) * size + (x + r)] = val;
            total += val;
        }
    const double mean = total / n;
    double peak = 0.0;
    for (int i = 0; i < n; ++i) {
        v[i] -= mean;
        peak = std::max(peak, std::fabs(v[i]));
    }
    if (!(peak > 0.0)) return set_err(nullptr, LOGFX_EINVAL, "degenerate mask");
    int e;
    std::frexp(peak, &e);
    const double u = std::ldexp(1.0, e - grid_bits);
    long long k[225], sum = 0;
    for (int i = 0; i < n; ++i) {
        k[i] = (long long)std::nearbyint(v[i] / u);
        sum += k[i];
    }
    k[r * size + r] -= sum;  // exact zero sum
    for (int i = 0; i < n; ++i) taps_out[i] = (float)((double)k[i] * u);
    if (unit_out) *unit_out = u;
    return LOGFX_OK;
}

int logfx_check_params(const logfx_image *img, const logfx_params *p, int32_t *path_out) {
    Plan pl;
    int rc = check_all(nullptr, img, p, pl);
    if (rc == LOGFX_OK && path_out) *path_out = pl.path;
    return rc;
}

static int run(logfx_ctx *ctx, const logfx_image *img, const logfx_params *p, uint8_t *out,
               double *const maps_L[2], double *const maps_Z[2], logfx_report *rep, void *stream) {
    if (!ctx) return set_err(nullptr, LOGFX_EINVAL, "ctx is NULL");
    ctx->err.clear();
    Plan pl;
    int rc = check_all(ctx, img, p, pl);
    if (rc != LOGFX_OK) return rc;
    const bool maps = maps_L != nullptr;
    if (!maps && !out) return set_err(ctx, LOGFX_EINVAL, "out is NULL");
    Geometry g;
    if ((rc = geometry(ctx, img, pl, g)) != LOGFX_OK) return rc;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return set_err(ctx, LOGFX_EDEVICE, "cannot select device %d", ctx->device);
    if ((rc = ensure_scratch(ctx, g.ntiles1, g.ntiles2)) != LOGFX_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    const bool timed = ctx->timing && !maps;
    if (timed) {
        if ((rc = timing_events(ctx, ctx->timed_calls, ev)) != LOGFX_OK) return rc;
        if ((e = hipEventRecord(ev[0], s)) != hipSuccess) return hip_err(ctx, e, "hipEventRecord");
    }
    const bool i32 = pl.path == LOGFX_PATH_INT32;
    e = i32 ? launch_p1<OrbitTapsI, int>(pl, g, ctx, img, p, maps_L, maps_Z, s)
            : launch_p1<OrbitTapsD, double>(pl, g, ctx, img, p, maps_L, maps_Z, s);
    if (e != hipSuccess) return hip_err(ctx, e, "pass-1 launch");
    if (maps) return LOGFX_OK;
    if (timed && (e = hipEventRecord(ev[1], s)) != hipSuccess) return hip_err(ctx, e, "hipEventRecord");

    FinalizeArgs f;
    std::memset(&f, 0, sizeof f);
    f.partials = ctx->partials;
    f.counts = ctx->counts1;
    f.ntiles = g.ntiles1;
    f.n = img->height * img->width;
    f.std_mode = p->std_mode;
    f.std_k = p->std_k;
    for (int slot = 0; slot < 2; ++slot) f.abs_thr[slot] = p->std_k / pl.mi[pl.order[slot]].unit;
    f.stats = ctx->stats;
    if ((e = launch_finalize(f, s)) != hipSuccess) return hip_err(ctx, e, "finalize launch");
    if (timed && (e = hipEventRecord(ev[2], s)) != hipSuccess) return hip_err(ctx, e, "hipEventRecord");

    e = i32 ? launch_p2<OrbitTapsI, int>(pl, g, ctx, img, p, out, s)
            : launch_p2<OrbitTapsD, double>(pl, g, ctx, img, p, out, s);
    if (e != hipSuccess) return hip_err(ctx, e, "pass-2 launch");
    if (timed) {
        if ((e = hipEventRecord(ev[3], s)) != hipSuccess) return hip_err(ctx, e, "hipEventRecord");
        ++ctx->timed_calls;
    }

    if (rep) {
        if ((rc = ensure_host(ctx, g.ntiles2)) != LOGFX_OK) return rc;
        if ((e = hipMemcpyAsync(ctx->h_stats, ctx->stats, sizeof(DevStats), hipMemcpyDeviceToHost,
                                s)) != hipSuccess ||
            (e = hipMemcpyAsync(ctx->h_counts2, ctx->counts2, (size_t)g.ntiles2 * 2 * sizeof(int),
                                hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return hip_err(ctx, e, "report copy");
        std::memset(rep, 0, sizeof *rep);
        rep->pixels = f.n;
        for (int slot = 0; slot < 2; ++slot) {
            const int u = pl.order[slot];
            const double unit = pl.mi[u].unit;
            rep->sigma_g[u] = ctx->h_stats->sigma[slot] * unit;
            rep->thresh[u] = ctx->h_stats->thresh[slot] * unit;
            rep->zc_count[u] = ctx->h_stats->zc[slot];
        }
        for (int t = 0; t < g.ntiles2; ++t) {
            rep->extracted += ctx->h_counts2[2 * t];
            rep->output += ctx->h_counts2[2 * t + 1];
        }
        rep->path = pl.path;
        rep->smoothed = p->smooth == LOGFX_SMOOTH_ALWAYS;
    }
    return LOGFX_OK;
}

int logfx_extract(logfx_ctx *ctx, const logfx_image *img, const logfx_params *p, uint8_t *out,
                  logfx_report *rep, void *stream) {
    return run(ctx, img, p, out, nullptr, nullptr, rep, stream);
}

int logfx_extract_maps(logfx_ctx *ctx, const logfx_image *img, const logfx_params *p, double *L1,
                       double *L2, double *Z1, double *Z2, void *stream) {
    double *L[2] = {L1, L2}, *Z[2] = {Z1, Z2};
    return run(ctx, img, p, nullptr, L, Z, nullptr, stream);
}

int logfx_timing_enable(logfx_ctx *ctx, int on) {
    if (!ctx) return set_err(nullptr, LOGFX_EINVAL, "ctx is NULL");
    ctx->timing = on != 0;
    ctx->timed_calls = 0;
    return LOGFX_OK;
}

int logfx_timing_read(logfx_ctx *ctx, double *ms_out, int64_t *calls_out) {
    if (!ctx || !ms_out) return set_err(ctx, LOGFX_EINVAL, "ctx or ms_out is NULL");
    ms_out[0] = ms_out[1] = ms_out[2] = 0.0;
    DeviceGuard dg(ctx->device);
    for (long long c = 0; c < ctx->timed_calls; ++c) {
        hipEvent_t *ev = &ctx->events[4 * c];
        hipError_t e = hipEventSynchronize(ev[3]);
        if (e != hipSuccess) return hip_err(ctx, e, "hipEventSynchronize");
        for (int k = 0; k < 3; ++k) {
            float ms = 0.0f;
            if ((e = hipEventElapsedTime(&ms, ev[k], ev[k + 1])) != hipSuccess)
                return hip_err(ctx, e, "hipEventElapsedTime");
            ms_out[k] += ms;
        }
    }
    if (calls_out) *calls_out = ctx->timed_calls;
    ctx->timed_calls = 0;
    return LOGFX_OK;
}

}  // extern "C"
