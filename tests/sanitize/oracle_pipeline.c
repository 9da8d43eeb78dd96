/* The CPU oracle (oracle/logfx_oracle.c) under AddressSanitizer and
 * UndefinedBehaviorSanitizer (built by tests/test_sanitizers.py): the whole
 * pipeline on degenerate and ragged shapes, both pixel types, every option,
 * one and several threads.  Checks only what any run must satisfy (binary
 * maps, finite statistics, equal results for any thread count); the
 * arithmetic itself is pinned by tests/test_oracle.py.  A sanitizer report
 * aborts the program. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int orc_log_mask(int size, double sigma, int grid_bits, float *taps, double *unit);
int orc_extract(const void *img, int dtype, long H, long W, long pitch, const float *taps1, int size1,
                const float *taps2, int size2, double zc_thresh, int std_mode, double std_k, double std5_max,
                int smooth, int median_size, uint8_t *F, uint8_t *E_out, double *L1o, double *L2o, double *Z1o,
                double *Z2o, double *S1o, double *S2o, double *stats, int nthreads);

static unsigned long long rng = 88172645463325252ull;
static unsigned next(void) {
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return (unsigned)(rng >> 11);
}

static int failures = 0;
#define EXPECT(c)                                                 \
    do {                                                          \
        if (!(c)) {                                               \
            fprintf(stderr, "%s:%d: %s\n", __FILE__, __LINE__, #c); \
            ++failures;                                           \
        }                                                         \
    } while (0)

int main(void) {
    float t5[25], t9[81], t3[9], t7[49];
    EXPECT(orc_log_mask(5, 0.8, 16, t5, NULL) == 0);
    EXPECT(orc_log_mask(9, 1.4, 16, t9, NULL) == 0);
    EXPECT(orc_log_mask(3, 0.5, 16, t3, NULL) == 0);
    EXPECT(orc_log_mask(7, 1.0, 23, t7, NULL) == 0);
    const long shapes[][3] = {{1, 1, 1}, {1, 37, 40}, {29, 1, 1}, {2, 2, 2}, {3, 200, 203},
                              {37, 53, 53}, {64, 65, 72}, {130, 9, 9}, {9, 131, 131}};
    const int nshapes = sizeof shapes / sizeof shapes[0];
    for (int s = 0; s < nshapes; ++s) {
        const long H = shapes[s][0], W = shapes[s][1], P = shapes[s][2];
        for (int dtype = 0; dtype < 2; ++dtype) {
            const long n = H * P;
            void *img = malloc((size_t)n * (dtype ? 2 : 1));
            for (long i = 0; i < n; ++i) {
                if (dtype) ((uint16_t *)img)[i] = (uint16_t)(next() & 2047);
                else ((uint8_t *)img)[i] = (uint8_t)(next() & 255);
            }
            for (int opt = 0; opt < 6; ++opt) {
                const float *a = opt == 3 ? t3 : t5, *b = opt == 4 ? t7 : t9;
                const int sa = opt == 3 ? 3 : 5, sb = opt == 4 ? 7 : 9;
                const double zc = opt == 1 ? 2.0 : 0.0, s5 = opt == 2 ? 0.5 : -1.0;
                const int mode = opt == 5, smooth = opt != 1, med = opt == 4 ? 3 : 5;
                uint8_t *F1 = malloc((size_t)(H * W)), *F3 = malloc((size_t)(H * W)), *E = malloc((size_t)(H * W));
                double *Z1 = malloc(sizeof(double) * H * W), *S2 = malloc(sizeof(double) * H * W);
                double st1[4], st3[4];
                EXPECT(orc_extract(img, dtype, H, W, P, a, sa, b, sb, zc, mode, mode ? 3.0 : 2.0, s5, smooth, med,
                                   F1, E, NULL, NULL, Z1, NULL, NULL, S2, st1, 1) == 0);
                EXPECT(orc_extract(img, dtype, H, W, P, a, sa, b, sb, zc, mode, mode ? 3.0 : 2.0, s5, smooth, med,
                                   F3, NULL, NULL, NULL, NULL, NULL, NULL, NULL, st3, 3) == 0);
                EXPECT(memcmp(F1, F3, (size_t)(H * W)) == 0);
                EXPECT(memcmp(st1, st3, sizeof st1) == 0);
                for (long i = 0; i < H * W; ++i) {
                    EXPECT(F1[i] <= 1 && E[i] <= 1);
                    EXPECT(Z1[i] >= 0.0 && isfinite(S2[i]));
                    if (failures > 20) return 1;
                }
                for (int k = 0; k < 4; ++k) EXPECT(isfinite(st1[k]) && st1[k] >= 0.0);
                free(F1); free(F3); free(E); free(Z1); free(S2);
            }
            free(img);
        }
    }
    /* refused arguments */
    uint8_t F[4];
    uint8_t px[4] = {1, 2, 3, 4};
    EXPECT(orc_extract(NULL, 0, 2, 2, 2, t5, 5, t9, 9, 0, 0, 2, -1, 1, 5, F, NULL, NULL, NULL, NULL, NULL, NULL,
                       NULL, NULL, 1) != 0);
    EXPECT(orc_extract(px, 0, 2, 2, 1, t5, 5, t9, 9, 0, 0, 2, -1, 1, 5, F, NULL, NULL, NULL, NULL, NULL, NULL,
                       NULL, NULL, 1) != 0);
    if (failures) fprintf(stderr, "%d failure(s)\n", failures);
    else printf("oracle pipeline: ok\n");
    return failures ? 1 : 0;
}
