// Host-only entry points of liblogfx under AddressSanitizer and
// UndefinedBehaviorSanitizer (built by tests/test_sanitizers.py; no GPU is
// used): mask construction over every size, sigma and grid, the argument and
// exactness checks on valid and invalid requests, and the calls that must
// fail before touching a device.  Exits 0 when every expectation holds; a
// sanitizer report aborts the program.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "logfx.h"

static int failures = 0;
#define EXPECT(c)                                                   \
    do {                                                            \
        if (!(c)) {                                                 \
            std::fprintf(stderr, "%s:%d: %s\n", __FILE__, __LINE__, #c); \
            ++failures;                                             \
        }                                                           \
    } while (0)

int main() {
    EXPECT(std::strstr(logfx_version(), "liblogfx") != nullptr);
    std::vector<float> m1(81), m2(81);
    double u = 0;
    // masks: every odd size up to 15, several sigmas and grids
    for (int size = 1; size <= 17; ++size)
        for (double sigma : {0.3, 0.8, 1.4, 3.0})
            for (int g : {1, 2, 8, 16, 23, 24}) {
                std::vector<float> t(size * size + 1, 0.0f);
                const int rc = logfx_make_log_mask(size, sigma, g, t.data(), &u);
                const bool ok = size % 2 == 1 && size <= 15 && size >= 3 && g >= 2 && g <= 23;
                if (size == 1) EXPECT(rc != LOGFX_OK);
                else EXPECT((rc == LOGFX_OK) == ok);
                if (rc == LOGFX_OK) {
                    double s = 0;
                    for (int i = 0; i < size * size; ++i) s += t[i];
                    EXPECT(s == 0.0);
                }
            }
    EXPECT(logfx_make_log_mask(5, 0.8, 16, nullptr, nullptr) == LOGFX_EINVAL);
    EXPECT(logfx_make_log_mask(5, NAN, 16, m1.data(), nullptr) == LOGFX_EINVAL);
    EXPECT(logfx_make_log_mask(5, 0.8, 16, m1.data(), nullptr) == LOGFX_OK);
    EXPECT(logfx_make_log_mask(9, 1.4, 16, m2.data(), nullptr) == LOGFX_OK);
    EXPECT(std::strlen(logfx_last_error(nullptr)) < 512);

    logfx_image img;
    std::memset(&img, 0, sizeof img);
    img.data = reinterpret_cast<const void *>(0x1000);   // never dereferenced
    img.dtype = LOGFX_U16;
    img.bits = 11;
    img.height = 100;
    img.width = 130;
    img.pitch = 130;
    logfx_params p;
    std::memset(&p, 0, sizeof p);
    p.mask[0] = {5, m1.data()};
    p.mask[1] = {9, m2.data()};
    p.std_k = 2.0;
    p.std5_max = -1.0;
    p.smooth = LOGFX_SMOOTH_ALWAYS;
    p.median_size = 5;
    int32_t path = -1;
    EXPECT(logfx_check_params(&img, &p, &path) == LOGFX_OK && path == LOGFX_PATH_INT32);
    // one field at a time made invalid
    struct Case { const char *what; void (*edit)(logfx_image &, logfx_params &); int want; };
    const Case cases[] = {
        {"height 0", [](logfx_image &i, logfx_params &) { i.height = 0; }, LOGFX_EINVAL},
        {"pitch < width", [](logfx_image &i, logfx_params &) { i.pitch = 10; }, LOGFX_EINVAL},
        {"dtype", [](logfx_image &i, logfx_params &) { i.dtype = 7; }, LOGFX_EINVAL},
        {"bits 17", [](logfx_image &i, logfx_params &) { i.bits = 17; }, LOGFX_EINVAL},
        {"bits 16: FP64 path", [](logfx_image &i, logfx_params &) { i.bits = 16; }, LOGFX_OK},
        {"median 4", [](logfx_image &, logfx_params &q) { q.median_size = 4; }, LOGFX_EINVAL},
        {"smooth 9", [](logfx_image &, logfx_params &q) { q.smooth = 9; }, LOGFX_EINVAL},
        {"std_k < 0", [](logfx_image &, logfx_params &q) { q.std_k = -1; }, LOGFX_EINVAL},
        {"std_k NaN", [](logfx_image &, logfx_params &q) { q.std_k = NAN; }, LOGFX_EINVAL},
        {"zc NaN", [](logfx_image &, logfx_params &q) { q.zc_thresh = NAN; }, LOGFX_EINVAL},
        {"std5 NaN", [](logfx_image &, logfx_params &q) { q.std5_max = NAN; }, LOGFX_EINVAL},
        {"flags", [](logfx_image &, logfx_params &q) { q.flags = 6; }, LOGFX_EINVAL},
        {"mask even", [](logfx_image &, logfx_params &q) { q.mask[0].size = 4; }, LOGFX_EINVAL},
        {"mask 11", [](logfx_image &, logfx_params &q) { q.mask[1].size = 11; }, LOGFX_EUNSUPPORTED},
        {"mask NULL", [](logfx_image &, logfx_params &q) { q.mask[0].taps = nullptr; }, LOGFX_EINVAL},
        {"cascade 7", [](logfx_image &, logfx_params &q) { q.median_cascade[0] = 7; }, LOGFX_EINVAL},
        {"cascade gap", [](logfx_image &, logfx_params &q) { q.median_cascade[1] = 3; }, LOGFX_EINVAL},
        {"region w/o gate", [](logfx_image &, logfx_params &q) { q.gate_region = 128; }, LOGFX_EINVAL},
        {"region < 0", [](logfx_image &, logfx_params &q) { q.gate_region = -1; }, LOGFX_EINVAL},
    };
    for (const Case &c : cases) {
        logfx_image i2 = img;
        logfx_params p2 = p;
        c.edit(i2, p2);
        const int rc = logfx_check_params(&i2, &p2, &path);
        if (rc != c.want) std::fprintf(stderr, "case %s: %d (%s)\n", c.what, rc, logfx_last_error(nullptr));
        EXPECT(rc == c.want);
    }
    EXPECT(logfx_check_params(nullptr, &p, &path) == LOGFX_EINVAL);
    EXPECT(logfx_check_params(&img, nullptr, &path) == LOGFX_EINVAL);
    // an asymmetric mask
    std::vector<float> asym(m1);
    asym[1] += asym[1] == 0.0f ? 1.0f : asym[1];
    logfx_params pa = p;
    pa.mask[0].taps = asym.data();
    EXPECT(logfx_check_params(&img, &pa, &path) == LOGFX_EUNSUPPORTED);
    // NULL contexts are refused before any device call
    uint8_t *out = reinterpret_cast<uint8_t *>(0x2000);
    EXPECT(logfx_extract(nullptr, &img, &p, out, nullptr, nullptr) == LOGFX_EINVAL);
    EXPECT(logfx_extract_batch(nullptr, 1, &img, &p, &out, nullptr, nullptr) == LOGFX_EINVAL);
    EXPECT(logfx_gate(nullptr, 1, &img, &p, nullptr, nullptr, nullptr) == LOGFX_EINVAL);
    EXPECT(logfx_set_option(nullptr, LOGFX_OPT_ROWS1, 64) == LOGFX_EINVAL);
    EXPECT(logfx_destroy(nullptr) == LOGFX_OK);
    // without a GPU the context cannot be made, and says why
    logfx_ctx *ctx = nullptr;
    const int rc = logfx_create(&ctx, 0);
    if (rc != LOGFX_OK) {
        EXPECT(ctx == nullptr && std::strlen(logfx_last_error(nullptr)) > 0);
    } else {
        logfx_destroy(ctx);
    }
    EXPECT(logfx_create(nullptr, 0) == LOGFX_EINVAL);
    if (failures) std::fprintf(stderr, "%d failure(s)\n", failures);
    else std::printf("host entry points: ok\n");
    return failures ? 1 : 0;
}
