/*
 * logfx_oracle.c -- TEST INFRASTRUCTURE, not part of the product.
 *
 * A plain, slow, obviously correct CPU implementation (FP64) of the feature
 * extraction pipeline of Tejaswi, Rao, Nair and Prasad, "GPU accelerated
 * automated feature extraction from satellite images" (arXiv:1304.3992):
 *
 *   image -> LoG(mask 1), LoG(mask 2)          (Sec. 3.1, eq. (1); Sec. 4.1)
 *         -> zero crossings + strength          (Sec. 3.2; Sec. 4; Sec. 4.1)
 *         -> local standard deviation test      (Sec. 3.3, eq. (2); Sec. 4.1)
 *         -> OR of the two extracted maps       (abstract; Sec. 4.1)
 *         -> optional hybrid median filter      (Sec. 3.4; abstract)
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this file's library.  It shares no code, header or table with the GPU
 * library; each side builds its own masks and the tests compare them.
 *
 * Every stage reads its input through clamp-to-edge indexing (the padding the
 * paper describes in Sec. 4.1 does not state its values; replicated edges are
 * the reading taken here).  Each function states the passage it follows.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fPIC -shared -pthread
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_U8 0
#define ORC_U16 1

static long clampl(long v, long lo, long hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* Pixel (y, x) of an image read with clamp-to-edge indexing. */
static double pix(const void *img, int dtype, long H, long W, long pitch, long y, long x)
{
    y = clampl(y, 0, H - 1);
    x = clampl(x, 0, W - 1);
    if (dtype == ORC_U8) return (double)((const uint8_t *)img)[y * pitch + x];
    return (double)((const uint16_t *)img)[y * pitch + x];
}

static double at(const double *a, long H, long W, long y, long x)
{
    return a[clampl(y, 0, H - 1) * W + clampl(x, 0, W - 1)];
}

/* ------------------------------------------------------------------------
 * Row-band threading helper (only used to time the oracle on all cores; the
 * result does not depend on the number of threads because every per-pixel
 * value is computed independently).
 * ---------------------------------------------------------------------- */
typedef void (*band_fn)(void *ctx, long y0, long y1);
typedef struct { band_fn fn; void *ctx; long y0, y1; } band_job;
static void *band_run(void *p) { band_job *j = (band_job *)p; j->fn(j->ctx, j->y0, j->y1); return NULL; }

static void run_bands(band_fn fn, void *ctx, long H, int nthreads)
{
    if (nthreads <= 1 || H < 2) { fn(ctx, 0, H); return; }
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    band_job jobs[256];
    for (int t = 0; t < nthreads; ++t) {
        jobs[t].fn = fn; jobs[t].ctx = ctx;
        jobs[t].y0 = H * t / nthreads; jobs[t].y1 = H * (t + 1) / nthreads;
        pthread_create(&th[t], NULL, band_run, &jobs[t]);
    }
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
}

/* ------------------------------------------------------------------------
 * Eq. (1), Sec. 3.1: LoG(x,y) = -1/(pi s^4) [1 - (x^2+y^2)/(2 s^2)] exp(-(x^2+y^2)/(2 s^2)).
 * ---------------------------------------------------------------------- */
double orc_log_value(double x, double y, double sigma)
{
    double q = (x * x + y * y) / (2.0 * sigma * sigma);
    return -1.0 / (M_PI * sigma * sigma * sigma * sigma) * (1.0 - q) * exp(-q);
}

/* Mask construction (reading of Sec. 3.1 and Sec. 4.1; the paper gives the
 * function and the window size but not how the sampled taps are made to sum
 * to zero or stored):
 *   1. sample eq. (1) at integer offsets of a size x size window (FP64);
 *   2. subtract the FP64 mean of the samples;
 *   3. snap every tap to the grid u = 2^(e + 1 - grid_bits), where
 *      2^e <= max|tap| < 2^(e+1), rounding half to even;
 *   4. subtract the integer sum of the snapped taps from the centre tap, so
 *      that the integer taps k sum to exactly zero;
 *   5. store k * u as float (exact for grid_bits <= 23).
 * Returns 0, or -1 on invalid arguments.  *unit receives u. */
int orc_log_mask(int size, double sigma, int grid_bits, float *taps, double *unit)
{
    if (size < 1 || size % 2 == 0 || size > 15 || !(sigma > 0) || grid_bits < 2 || grid_bits > 23)
        return -1;
    int r = size / 2, n = size * size;
    double v[225];
    double sum = 0.0;
    for (int dy = -r; dy <= r; ++dy)
        for (int dx = -r; dx <= r; ++dx) {
            double t = orc_log_value((double)dx, (double)dy, sigma);
            v[(dy + r) * size + (dx + r)] = t;
            sum += t;
        }
    double mean = sum / n;
    double amax = 0.0;
    for (int i = 0; i < n; ++i) {
        v[i] -= mean;
        if (fabs(v[i]) > amax) amax = fabs(v[i]);
    }
    if (!(amax > 0)) return -1;
    int e2;
    frexp(amax, &e2);               /* amax = m * 2^e2, 0.5 <= m < 1, so e = e2 - 1 */
    double u = ldexp(1.0, e2 - grid_bits);
    long long k[225], ksum = 0;
    for (int i = 0; i < n; ++i) {
        k[i] = (long long)nearbyint(v[i] / u);
        ksum += k[i];
    }
    k[r * size + r] -= ksum;
    for (int i = 0; i < n; ++i) taps[i] = (float)((double)k[i] * u);
    if (unit) *unit = u;
    return 0;
}

/* ------------------------------------------------------------------------
 * LoG response, Sec. 4.1: the mask is applied to every pixel with its
 * size x size neighbourhood.  Correlation with clamp-to-edge borders; for the
 * symmetric masks of eq. (1) this equals convolution.  FP64 sum in row-major
 * tap order.
 * ---------------------------------------------------------------------- */
typedef struct {
    const void *img; int dtype; long H, W, pitch; const float *taps; int size; double *L;
} log_ctx;

static void log_band(void *p, long y0, long y1)
{
    log_ctx *c = (log_ctx *)p;
    int r = c->size / 2;
    for (long y = y0; y < y1; ++y)
        for (long x = 0; x < c->W; ++x) {
            double s = 0.0;
            for (int i = 0; i < c->size; ++i)
                for (int j = 0; j < c->size; ++j)
                    s += (double)c->taps[i * c->size + j] *
                         pix(c->img, c->dtype, c->H, c->W, c->pitch, y + i - r, x + j - r);
            c->L[y * c->W + x] = s;
        }
}

void orc_log_response(const void *img, int dtype, long H, long W, long pitch,
                      const float *taps, int size, double *L, int nthreads)
{
    log_ctx c = {img, dtype, H, W, pitch, taps, size, L};
    run_bands(log_band, &c, H, nthreads);
}

/* ------------------------------------------------------------------------
 * Zero crossings, Sec. 3.2 and Sec. 4 (four neighbours up/down/left/right).
 * Reading taken where the text is silent:
 *  - p with L(p) != 0 is a crossing if SOME neighbour q has the opposite sign
 *    and p has the smaller |L| of the pair; on a tie the negative pixel is
 *    the crossing (each opposite-sign pair marks exactly one pixel);
 *  - p with L(p) == 0 is a crossing if its left/right or its up/down
 *    neighbours have opposite signs;
 *  - strength c(p) = max - min of L over p and its four neighbours (at a
 *    crossing the largest value is positive and the smallest negative, so
 *    this is the span across zero that Sec. 3.2 thresholds);
 *  - Z(p) = c(p) if p is a crossing and c(p) > zc_thresh, else 0.
 * ---------------------------------------------------------------------- */
static int opposite(double a, double b) { return (a < 0 && b > 0) || (a > 0 && b < 0); }

typedef struct { const double *L; long H, W; double thr; double *Z; } zc_ctx;

static void zc_band(void *p, long y0, long y1)
{
    zc_ctx *c = (zc_ctx *)p;
    long H = c->H, W = c->W;
    for (long y = y0; y < y1; ++y)
        for (long x = 0; x < W; ++x) {
            double a = at(c->L, H, W, y, x);
            double nb[4] = {at(c->L, H, W, y - 1, x), at(c->L, H, W, y + 1, x),
                            at(c->L, H, W, y, x - 1), at(c->L, H, W, y, x + 1)};
            int is = 0;
            if (a != 0.0) {
                for (int k = 0; k < 4; ++k) {
                    double b = nb[k];
                    if (!opposite(a, b)) continue;
                    if (fabs(a) < fabs(b) || (fabs(a) == fabs(b) && a < 0)) is = 1;
                }
            } else {
                is = opposite(nb[2], nb[3]) || opposite(nb[0], nb[1]);
            }
            double mx = a, mn = a;
            for (int k = 0; k < 4; ++k) {
                if (nb[k] > mx) mx = nb[k];
                if (nb[k] < mn) mn = nb[k];
            }
            double cst = mx - mn;
            c->Z[y * W + x] = (is && cst > c->thr) ? cst : 0.0;
        }
}

void orc_zero_cross(const double *L, long H, long W, double zc_thresh, double *Z, int nthreads)
{
    zc_ctx c = {L, H, W, zc_thresh, Z};
    run_bands(zc_band, &c, H, nthreads);
}

/* ------------------------------------------------------------------------
 * Eq. (2), Sec. 3.3: unbiased sample standard deviation
 *     s = sqrt( sum (a - m)^2 / (N - 1) ),  m = mean of the N values.
 * Global form over a whole map (compensated Neumaier sums, two passes).
 * N <= 1 gives 0.
 * ---------------------------------------------------------------------- */
typedef struct { double s, c; } neu;
static void neu_add(neu *a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}

double orc_global_std(const double *Z, long n)
{
    if (n <= 1) return 0.0;
    neu s1 = {0, 0};
    for (long i = 0; i < n; ++i) neu_add(&s1, Z[i]);
    double mean = (s1.s + s1.c) / (double)n;
    neu s2 = {0, 0};
    for (long i = 0; i < n; ++i) { double d = Z[i] - mean; neu_add(&s2, d * d); }
    return sqrt((s2.s + s2.c) / (double)(n - 1));
}

/* Local form: eq. (2) over the clamped win x win window around each pixel
 * (Sec. 4.1 uses 5 x 5 and then 3 x 3 windows). */
typedef struct { const double *Z; long H, W; int win; double *S; } lstd_ctx;

static void lstd_band(void *p, long y0, long y1)
{
    lstd_ctx *c = (lstd_ctx *)p;
    int r = c->win / 2, cnt = c->win * c->win;
    double v[225];
    for (long y = y0; y < y1; ++y)
        for (long x = 0; x < c->W; ++x) {
            int k = 0;
            double sum = 0.0;
            for (int dy = -r; dy <= r; ++dy)
                for (int dx = -r; dx <= r; ++dx) {
                    v[k] = at(c->Z, c->H, c->W, y + dy, x + dx);
                    sum += v[k++];
                }
            double m = sum / cnt, ss = 0.0;
            for (int i = 0; i < cnt; ++i) ss += (v[i] - m) * (v[i] - m);
            c->S[y * c->W + x] = sqrt(ss / (cnt - 1));
        }
}

void orc_local_std(const double *Z, long H, long W, int win, double *S, int nthreads)
{
    lstd_ctx c = {Z, H, W, win, S};
    run_bands(lstd_band, &c, H, nthreads);
}

/* ------------------------------------------------------------------------
 * Hybrid median filter, Sec. 3.4: two subgroups of the win x win
 * neighbourhood -- the pixels parallel to the axes (the "+" through the
 * centre) and the pixels at 45 degrees (the "x" through the centre), the
 * centre counted once in each -- are ranked, and the output is the median of
 * {median(+), median(x), centre}.  Clamped borders.  Works on any 8-bit
 * values (the pipeline applies it to the 0/1 extracted map).
 * ---------------------------------------------------------------------- */
static void sort_u8(uint8_t *a, int n)
{
    for (int i = 1; i < n; ++i) {
        uint8_t v = a[i];
        int j = i - 1;
        while (j >= 0 && a[j] > v) { a[j + 1] = a[j]; --j; }
        a[j + 1] = v;
    }
}

static uint8_t at8(const uint8_t *a, long H, long W, long y, long x)
{
    return a[clampl(y, 0, H - 1) * W + clampl(x, 0, W - 1)];
}

typedef struct { const uint8_t *E; long H, W; int win; uint8_t *F; } hm_ctx;

static void hm_band(void *p, long y0, long y1)
{
    hm_ctx *c = (hm_ctx *)p;
    int r = c->win / 2;
    uint8_t plus[32], cross[32];
    for (long y = y0; y < y1; ++y)
        for (long x = 0; x < c->W; ++x) {
            int np = 0, nc = 0;
            plus[np++] = at8(c->E, c->H, c->W, y, x);
            cross[nc++] = at8(c->E, c->H, c->W, y, x);
            for (int d = 1; d <= r; ++d) {
                plus[np++] = at8(c->E, c->H, c->W, y - d, x);
                plus[np++] = at8(c->E, c->H, c->W, y + d, x);
                plus[np++] = at8(c->E, c->H, c->W, y, x - d);
                plus[np++] = at8(c->E, c->H, c->W, y, x + d);
                cross[nc++] = at8(c->E, c->H, c->W, y - d, x - d);
                cross[nc++] = at8(c->E, c->H, c->W, y - d, x + d);
                cross[nc++] = at8(c->E, c->H, c->W, y + d, x - d);
                cross[nc++] = at8(c->E, c->H, c->W, y + d, x + d);
            }
            sort_u8(plus, np);
            sort_u8(cross, nc);
            uint8_t three[3] = {plus[np / 2], cross[nc / 2], at8(c->E, c->H, c->W, y, x)};
            sort_u8(three, 3);
            c->F[y * c->W + x] = three[1];
        }
}

void orc_hybrid_median(const uint8_t *E, long H, long W, int win, uint8_t *F, int nthreads)
{
    hm_ctx c = {E, H, W, win, F};
    run_bands(hm_band, &c, H, nthreads);
}

/* ------------------------------------------------------------------------
 * The whole pipeline, Sec. 4.1 (Fig. 1 flow): two LoG responses, zero
 * crossings on each, the standard-deviation extraction on each, the OR of
 * the two extracted maps, and optionally the hybrid median.
 *
 * Standard-deviation stage (reading of Sec. 4.1): per mask j,
 *   T_j = std_k * sigma_g(Z_j)   (std_mode 0: relative to the global
 *                                 standard deviation of the Z map), or
 *   T_j = std_k                  (std_mode 1: absolute);
 *   E_j(p) = [s3(p) > T_j], with s3 the eq. (2) deviation of Z_j over the
 *   clamped 3 x 3 window; if std5_max >= 0 the 5 x 5 deviation must also
 *   exceed std5_max (the paper's 5 x 5 first stage).
 * E = E_1 OR E_2;  F = hybrid_median(E) if smooth, else E.
 *
 * Optional outputs (NULL to skip): L1, L2, Z1, Z2, S1, S2 (3 x 3 local std),
 * E.  stats[0..3] receives sigma_g(Z1), sigma_g(Z2), T_1, T_2.
 * ---------------------------------------------------------------------- */
int orc_extract(const void *img, int dtype, long H, long W, long pitch,
                const float *taps1, int size1, const float *taps2, int size2,
                double zc_thresh, int std_mode, double std_k, double std5_max,
                int smooth, int median_size,
                uint8_t *F, uint8_t *E_out, double *L1o, double *L2o, double *Z1o, double *Z2o,
                double *S1o, double *S2o, double *stats, int nthreads)
{
    if (!img || !F || H < 1 || W < 1 || pitch < W) return -1;
    long n = H * W;
    const float *taps[2] = {taps1, taps2};
    int sizes[2] = {size1, size2};
    double *outL[2] = {L1o, L2o}, *outZ[2] = {Z1o, Z2o}, *outS[2] = {S1o, S2o};
    double *L = (double *)malloc(sizeof(double) * n);
    double *Z = (double *)malloc(sizeof(double) * n);
    double *S3 = (double *)malloc(sizeof(double) * n);
    double *S5 = std5_max >= 0 ? (double *)malloc(sizeof(double) * n) : NULL;
    uint8_t *E = (uint8_t *)calloc(n, 1);
    if (!L || !Z || !S3 || !E || (std5_max >= 0 && !S5)) {
        free(L); free(Z); free(S3); free(S5); free(E);
        return -2;
    }
    for (int j = 0; j < 2; ++j) {
        orc_log_response(img, dtype, H, W, pitch, taps[j], sizes[j], L, nthreads);
        orc_zero_cross(L, H, W, zc_thresh, Z, nthreads);
        double sg = orc_global_std(Z, n);
        double T = std_mode == 0 ? std_k * sg : std_k;
        orc_local_std(Z, H, W, 3, S3, nthreads);
        if (S5) orc_local_std(Z, H, W, 5, S5, nthreads);
        for (long i = 0; i < n; ++i) {
            int e = S3[i] > T;
            if (S5) e = e && (S5[i] > std5_max);
            E[i] |= (uint8_t)e;
        }
        if (stats) { stats[j] = sg; stats[2 + j] = T; }
        if (outL[j]) memcpy(outL[j], L, sizeof(double) * n);
        if (outZ[j]) memcpy(outZ[j], Z, sizeof(double) * n);
        if (outS[j]) memcpy(outS[j], S3, sizeof(double) * n);
    }
    if (smooth) orc_hybrid_median(E, H, W, median_size, F, nthreads);
    else memcpy(F, E, n);
    if (E_out) memcpy(E_out, E, n);
    free(L); free(Z); free(S3); free(S5); free(E);
    return 0;
}
