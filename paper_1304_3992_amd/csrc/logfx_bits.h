// Bit-sliced logic of the binary hybrid median (Sec. 3.4).  Every bit of a
// word is one pixel, so one logic operation treats a whole word of pixels.
// Plain C++ with no GPU types, so that a host test can check the logic
// against the median's definition on every input pattern.
#pragma once

#if defined(__HIP__)
#define LOGFX_HD __host__ __device__
#else
#define LOGFX_HD
#endif

namespace logfx {
namespace kern {

// Full adder: a + b + c = s + 2 cy.
template <class T>
LOGFX_HD inline void fadd(T a, T b, T c, T &s, T &cy) {
    const T t = a ^ b;
    s = t ^ c;
    cy = (t & c) | (~t & a);
}
// [count >= 2] and [count >= 3] of four pixels.
template <class T>
LOGFX_HD inline void at_least_2_3_of_4(const T (&v)[4], T &g2, T &g3) {
    T s1, c1;
    fadd(v[0], v[1], v[2], s1, c1);
    const T s = s1 ^ v[3], c2 = s1 & v[3];   // count = s + 2 (c1 + c2)
    g2 = c1 | c2;
    g3 = (c1 & c2) | (g2 & s);
}
// [count >= 4] and [count >= 5] of eight pixels.
template <class T>
LOGFX_HD inline void at_least_4_5_of_8(const T (&v)[8], T &g4, T &g5) {
    T s1, c1, s2, c2, s3, c3;
    fadd(v[0], v[1], v[2], s1, c1);
    fadd(v[3], v[4], v[5], s2, c2);
    fadd(v[6], v[7], s1, s3, c3);
    const T s = s2 ^ s3, c4 = s2 & s3;       // count = s + 2 (c1 + c2 + c3 + c4)
    const T a12 = c1 & c2, a34 = c3 & c4, o12 = c1 | c2, o34 = c3 | c4;
    g4 = a12 | a34 | (o12 & o34);            // at least two carries
    g5 = (a12 & o34) | (a34 & o12) | (g4 & s);
}
// Hybrid median (Sec. 3.4) of an M x M window of binary pixels: c is the
// centre, p the other 2M - 2 pixels of the "+" subgroup (centre row and
// column), x those of the "x" subgroup (the diagonals).  With the centre
// in both subgroups of 2M - 1 pixels, a subgroup's median is 1 iff it
// holds at least M ones, so the median of {median(+), median(x), c} is:
// for c = 1, at least M - 1 ones among the others of either subgroup; for
// c = 0, at least M ones among the others of both.
template <int M, class T>
LOGFX_HD inline T hybrid_median_bits(T c, const T (&p)[2 * M - 2], const T (&x)[2 * M - 2]) {
    static_assert(M == 3 || M == 5, "median window 3 or 5");
    T p1, p0, x1, x0;
    if constexpr (M == 3) {
        at_least_2_3_of_4(p, p1, p0);
        at_least_2_3_of_4(x, x1, x0);
    } else {
        at_least_4_5_of_8(p, p1, p0);
        at_least_4_5_of_8(x, x1, x0);
    }
    return (c & (p1 | x1)) | (~c & p0 & x0);
}
}  // namespace kern
}  // namespace logfx
