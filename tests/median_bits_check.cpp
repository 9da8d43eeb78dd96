// Host check of the bit-sliced hybrid median logic (logfx_bits.h) against
// the definition of Sec. 3.4: the median of {median of the "+" subgroup,
// median of the "x" subgroup, centre}, both subgroups holding the centre.
// Every pattern of the pixels the subgroups read is tried (2^9 for the 3x3
// window, 2^17 for the 5x5), 64 patterns per 64-bit word and 32 per 32-bit
// word, so that each bit position of a word is exercised.  Exit status 0
// when all agree.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "logfx_bits.h"

using logfx::kern::hybrid_median_bits;

static int median(std::vector<int> v) {
    std::sort(v.begin(), v.end());
    return v[v.size() / 2];
}

// Pixels of the window that the subgroups read: the centre, then the "+"
// offsets, then the "x" offsets.
struct Off { int r, c; };

template <int M>
static std::vector<Off> layout() {
    const int h = M / 2;
    std::vector<Off> v = {{0, 0}};
    for (int d = 1; d <= h; ++d) { v.push_back({0, -d}); v.push_back({0, d}); v.push_back({-d, 0}); v.push_back({d, 0}); }
    for (int d = 1; d <= h; ++d) { v.push_back({-d, -d}); v.push_back({-d, d}); v.push_back({d, -d}); v.push_back({d, d}); }
    return v;
}

template <int M, class T>
static long check() {
    constexpr int K = 2 * M - 2;   // other pixels per subgroup
    const std::vector<Off> L = layout<M>();
    const int n = (int)L.size();   // 1 + 2K
    const long total = 1L << n;
    constexpr int B = 8 * sizeof(T);
    long bad = 0;
    for (long base = 0; base < total; base += B) {
        T c = 0, p[K] = {}, x[K] = {};
        int want[B];
        for (int b = 0; b < B; ++b) {
            const long pat = (base + b) % total;
            auto px = [&](int i) { return (int)((pat >> i) & 1); };
            std::vector<int> plus = {px(0)}, diag = {px(0)};
            for (int i = 0; i < K; ++i) plus.push_back(px(1 + i));
            for (int i = 0; i < K; ++i) diag.push_back(px(1 + K + i));
            want[b] = median({median(plus), median(diag), px(0)});
            c |= (T)px(0) << b;
            for (int i = 0; i < K; ++i) {
                p[i] |= (T)px(1 + i) << b;
                x[i] |= (T)px(1 + K + i) << b;
            }
        }
        const T f = hybrid_median_bits<M>(c, p, x);
        for (int b = 0; b < B; ++b) bad += (int)((f >> b) & 1) != want[b];
    }
    std::printf("M=%d, %d-bit words: %ld patterns, %ld mismatches\n", M, B, total, bad);
    return bad;
}

int main() {
    long bad = check<3, uint32_t>() + check<3, uint64_t>() + check<5, uint32_t>() + check<5, uint64_t>();
    return bad == 0 ? 0 : 1;
}
