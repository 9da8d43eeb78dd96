"""Test infrastructure: an exact-rational brute-force version of the pipeline.

Independent of ``logfx_oracle.c`` (written separately, in Python, with
``fractions.Fraction`` so that nothing is rounded).  It is used only on tiny
images to pin the C oracle.  Same readings of the paper as the oracle:

* clamp-to-edge indexing at every stage (Sec. 4.1 pads without giving values);
* LoG response = correlation of the mask with the image (Sec. 4.1);
* zero crossing on the four neighbours (Sec. 3.2): a non-zero pixel is a
  crossing when a neighbour of opposite sign has a larger magnitude, ties
  going to the negative pixel; a zero pixel is a crossing when its
  left/right or up/down neighbours have opposite signs; the strength is the
  range of the five values and must exceed the threshold;
* eq. (2) (Sec. 3.3): unbiased standard deviation.  The threshold test
  s > T is decided exactly as s^2 > T^2 (both sides are non-negative);
* hybrid median (Sec. 3.4): median of {median(+), median(x), centre}.
"""
from __future__ import annotations

from fractions import Fraction


def _clamp(v, lo, hi):
    return lo if v < lo else hi if v > hi else v


def _get(a, y, x):
    H, W = len(a), len(a[0])
    return a[_clamp(y, 0, H - 1)][_clamp(x, 0, W - 1)]


def log_response(img, taps):
    """img: list of lists of ints; taps: 2-D sequence of floats (exactly
    converted).  Returns exact Fractions."""
    size = len(taps)
    r = size // 2
    T = [[Fraction(float(t)) for t in row] for row in taps]
    H, W = len(img), len(img[0])
    out = [[Fraction(0)] * W for _ in range(H)]
    for y in range(H):
        for x in range(W):
            acc = Fraction(0)
            for dy in range(-r, r + 1):
                for dx in range(-r, r + 1):
                    acc += T[dy + r][dx + r] * int(_get(img, y + dy, x + dx))
            out[y][x] = acc
    return out


def _sign(v):
    return (v > 0) - (v < 0)


def zc_pixel(c, up, down, left, right, thresh=Fraction(0)):
    """Zero-crossing value of one 5-point stencil (centre c).  Returns the
    strength if the centre is a crossing above ``thresh``, else 0."""
    nbrs = (up, down, left, right)
    crossing = False
    if c != 0:
        for q in nbrs:
            if _sign(q) == -_sign(c) and q != 0:
                if abs(c) < abs(q) or (abs(c) == abs(q) and c < 0):
                    crossing = True
    else:
        crossing = (_sign(left) * _sign(right) < 0) or (_sign(up) * _sign(down) < 0)
    strength = max((c,) + nbrs) - min((c,) + nbrs)
    return strength if (crossing and strength > thresh) else 0


def zero_cross(L, thresh=0):
    th = Fraction(thresh)
    H, W = len(L), len(L[0])
    return [[Fraction(zc_pixel(L[y][x], _get(L, y - 1, x), _get(L, y + 1, x),
                               _get(L, y, x - 1), _get(L, y, x + 1), th))
             for x in range(W)] for y in range(H)]


def variance(values):
    """Unbiased variance of a list of Fractions (eq. (2) squared); 0 for one value."""
    n = len(values)
    if n <= 1:
        return Fraction(0)
    m = sum(values, Fraction(0)) / n
    return sum(((v - m) ** 2 for v in values), Fraction(0)) / (n - 1)


def local_var(Z, win):
    r = win // 2
    H, W = len(Z), len(Z[0])
    return [[variance([_get(Z, y + dy, x + dx) for dy in range(-r, r + 1) for dx in range(-r, r + 1)])
             for x in range(W)] for y in range(H)]


def median(values):
    s = sorted(values)
    return s[len(s) // 2]


def hybrid_median(E, win=5):
    r = win // 2
    H, W = len(E), len(E[0])
    out = [[0] * W for _ in range(H)]
    for y in range(H):
        for x in range(W):
            plus = [_get(E, y, x)] + [_get(E, y + d * sy, x + d * sx) for d in range(1, r + 1)
                                      for (sy, sx) in ((-1, 0), (1, 0), (0, -1), (0, 1))]
            cross = [_get(E, y, x)] + [_get(E, y + d * sy, x + d * sx) for d in range(1, r + 1)
                                       for (sy, sx) in ((-1, -1), (-1, 1), (1, -1), (1, 1))]
            out[y][x] = median([median(plus), median(cross), _get(E, y, x)])
    return out


def extract(img, taps1, taps2, zc_thresh=0.0, std_mode=0, std_k=2.0, std5_max=-1.0,
            smooth=True, median_size=5):
    """Exact pipeline.  Returns dict with F, E (lists of 0/1), L1, L2, Z1, Z2
    (Fractions), V1, V2 (exact 3x3 variances), T2 (exact squared thresholds)."""
    H, W = len(img), len(img[0])
    n = H * W
    out = {}
    E = [[0] * W for _ in range(H)]
    k = Fraction(float(std_k))
    for j, taps in ((1, taps1), (2, taps2)):
        L = log_response(img, taps)
        Z = zero_cross(L, zc_thresh)
        gvar = variance([Z[y][x] for y in range(H) for x in range(W)]) if n > 1 else Fraction(0)
        T2 = k * k * gvar if std_mode == 0 else k * k
        V3 = local_var(Z, 3)
        V5 = local_var(Z, 5) if std5_max >= 0 else None
        t5 = Fraction(float(std5_max)) ** 2 if std5_max >= 0 else None
        for y in range(H):
            for x in range(W):
                e = V3[y][x] > T2
                if V5 is not None:
                    e = e and V5[y][x] > t5
                if e:
                    E[y][x] = 1
        out[f"L{j}"], out[f"Z{j}"], out[f"V{j}"], out[f"T2_{j}"] = L, Z, V3, T2
    out["E"] = E
    out["F"] = hybrid_median(E, median_size) if smooth else [row[:] for row in E]
    return out
