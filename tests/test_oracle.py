"""Pins of the CPU oracle against the paper and the mathematics (no GPU).

Each test names the passage it pins.  None of them re-types the oracle's own
formula: they use closed forms, library routines (scipy / numpy), invariants,
and an independent exact-rational brute force on tiny images.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.ndimage as ndi
from numpy.lib.stride_tricks import sliding_window_view

import oracle
from oracle import brute
from paper_1304_3992_amd import scenes

MASKS = [(3, 0.5), (5, 0.8), (7, 1.0), (9, 1.4), (11, 2.0)]


# ---------------------------------------------------------------- eq. (1)
@pytest.mark.parametrize("sigma", [0.5, 0.8, 1.4, 3.0])
def test_eq1_is_laplacian_of_unit_gaussian(sigma):
    """Eq. (1) must equal the Laplacian of the normalised 2-D Gaussian
    G = exp(-r^2 / 2 s^2) / (2 pi s^2): checked by central differences, which
    pins the sign, the -1/(pi s^4) factor and the exponent."""
    def G(x, y):
        return math.exp(-(x * x + y * y) / (2 * sigma * sigma)) / (2 * math.pi * sigma * sigma)
    h = 1e-3 * sigma
    for (x, y) in [(0, 0), (0.3, 0.1), (1.0, 0.0), (1.5, -0.7), (2.5, 2.0)]:
        lap = (G(x + h, y) + G(x - h, y) + G(x, y + h) + G(x, y - h) - 4 * G(x, y)) / (h * h)
        assert oracle.log_value(x, y, sigma) == pytest.approx(lap, rel=1e-5, abs=1e-9)


@pytest.mark.parametrize("size,sigma", MASKS)
@pytest.mark.parametrize("bits", [12, 16, 23])
def test_mask_zero_sum_symmetry_and_grid(size, sigma, bits):
    """Mask construction (reading of Sec. 3.1 / 4.1): exact zero sum, the
    eight symmetries of the square grid, every tap an integer multiple of the
    grid unit, off-centre taps within half a unit of the mean-removed eq. (1)
    samples and the centre within (n/2 + 1) units."""
    taps, u = oracle.log_mask(size, sigma, bits)
    k = taps.astype(np.float64) / u
    assert np.array_equal(k, np.round(k)), "taps are not on the grid"
    k = k.astype(np.int64)
    assert k.sum() == 0
    for t in (k.T, k[::-1], k[:, ::-1]):
        assert np.array_equal(t, k)
    r = size // 2
    ys, xs = np.mgrid[-r:r + 1, -r:r + 1]
    samples = np.vectorize(lambda x, y: oracle.log_value(x, y, sigma))(xs, ys)
    samples -= samples.mean()
    err = np.abs(k * u - samples)
    centre = err[r, r]
    err[r, r] = 0
    assert err.max() <= 0.5 * u * (1 + 1e-9)
    assert centre <= (size * size / 2 + 1) * u
    assert 2 ** (bits - 1) <= np.abs(k).max() <= 2 ** bits + size * size


def test_mask_rejects_bad_requests():
    for args in [(4, 1.0), (0, 1.0), (17, 1.0), (5, 0.0), (5, -1.0)]:
        with pytest.raises(ValueError):
            oracle.log_mask(*args)


# ---------------------------------------------------------------- LoG (Sec. 4.1)
def _masks(s1=5, g1=0.8, s2=9, g2=1.4, bits=16):
    return oracle.log_mask(s1, g1, bits)[0], oracle.log_mask(s2, g2, bits)[0]


@pytest.mark.parametrize("dtype,maxv", [(np.uint8, 255), (np.uint16, 2047), (np.uint16, 65535)])
@pytest.mark.parametrize("size,sigma", [(5, 0.8), (9, 1.4)])
def test_log_matches_scipy_correlate_nearest(dtype, maxv, size, sigma):
    """Clamp-to-edge correlation is scipy's mode='nearest'; with grid masks
    both sums are exact, so they must agree bit for bit."""
    rng = np.random.default_rng(7)
    img = rng.integers(0, maxv + 1, size=(37, 53)).astype(dtype)
    for bits in (16, 23):
        taps, _ = oracle.log_mask(size, sigma, bits)
        ref = ndi.correlate(img.astype(np.float64), taps.astype(np.float64), mode="nearest")
        assert np.array_equal(oracle.log_response(img, taps), ref)


def test_log_constant_offset_gain_and_ramp():
    """Zero-sum masks: a constant image gives 0, adding a constant changes
    nothing, scaling scales exactly, and a linear ramp gives 0 wherever the
    window does not reach the border (the discrete Laplacian of a plane)."""
    t1, t2 = _masks()
    for taps in (t1, t2):
        r = taps.shape[0] // 2
        const = np.full((20, 30), 123, np.uint8)
        assert not oracle.log_response(const, taps).any()
        rng = np.random.default_rng(3)
        img = rng.integers(0, 200, size=(24, 31)).astype(np.uint16)
        base = oracle.log_response(img, taps)
        assert np.array_equal(oracle.log_response(img + 55, taps), base)
        assert np.array_equal(oracle.log_response(img * 3, taps), 3 * base)
        yy, xx = np.mgrid[0:40, 0:50]
        ramp = (3 * xx + 2 * yy + 5).astype(np.uint16)
        Lr = oracle.log_response(ramp, taps)
        assert not Lr[r:-r, r:-r].any()


# ---------------------------------------------------------------- zero crossings (Sec. 3.2)
def test_zero_crossing_exhaustive_stencils():
    """All 5^5 five-point stencils with values in {-2..2}, oracle vs the
    independent brute force (Sec. 3.2 rule with the tie and zero readings)."""
    vals = [-2, -1, 0, 1, 2]
    cases = [(c, u, d, l, r) for c in vals for u in vals for d in vals for l in vals for r in vals]
    n = len(cases)
    L = np.zeros((3, 3 * n), np.float64)
    for i, (c, u, d, l, r) in enumerate(cases):
        b = 3 * i
        L[1, b + 1] = c
        L[0, b + 1] = u
        L[2, b + 1] = d
        L[1, b] = l
        L[1, b + 2] = r
    Z = oracle.zero_cross(L)
    for i, (c, u, d, l, r) in enumerate(cases):
        assert Z[1, 3 * i + 1] == brute.zc_pixel(c, u, d, l, r), (c, u, d, l, r)


def test_zero_crossing_threshold():
    """The strength must exceed the threshold (strict)."""
    L = np.array([[0, 0, 0], [3, -1, 0], [0, 0, 0]], np.float64)
    # centre -1, neighbours 0,0,3,0 -> crossing with strength 4
    assert oracle.zero_cross(L, 0.0)[1, 1] == 4
    assert oracle.zero_cross(L, 3.999)[1, 1] == 4
    assert oracle.zero_cross(L, 4.0)[1, 1] == 0


def test_zero_crossing_dihedral_invariance():
    rng = np.random.default_rng(11)
    L = rng.integers(-3, 4, size=(17, 17)).astype(np.float64)
    Z = oracle.zero_cross(L)
    for f in (np.transpose, np.flipud, np.fliplr, lambda a: np.rot90(a, 1)):
        assert np.array_equal(oracle.zero_cross(np.ascontiguousarray(f(L))), f(Z))


def _tail_sums(taps):
    """T(j) = sum over dx >= j of the column sums of the mask (exact)."""
    s = taps.shape[0]
    r = s // 2
    C = [sum(Fraction(float(taps[i, j])) for i in range(s)) for j in range(s)]
    return {j: sum(C[r + d] for d in range(j, r + 1)) for j in range(1, r + 2)}


@pytest.mark.parametrize("bits", [16, 23])
def test_step_edge_worked_example(bits):
    """Worked example: a vertical step a | b (b > a) at column c.  The LoG
    response is +(b-a) T(k+1) at column c-1-k and -(b-a) T(k+1) at column
    c+k, so exactly one column of crossings appears, at x = c (tie between c-1
    and c goes to the negative side), with strength (b-a)(T(1) + max(T(1),
    T(2))).  The global deviation is then sqrt(H z0^2 (1 - 1/W) / (HW - 1)),
    the 3x3 deviation is z0 / 2 on columns c-1..c+1 and 0 elsewhere, so with
    k = 2 exactly those three columns are extracted, and the hybrid median
    keeps the band."""
    H, W, c, a, b = 32, 64, 20, 40, 200
    img = np.full((H, W), a, np.uint8)
    img[:, c:] = b
    t1, t2 = _masks(bits=bits)
    for taps in (t1, t2):
        T = _tail_sums(taps)
        assert all(T[j] > 0 for j in range(1, taps.shape[0] // 2 + 1))
        L = oracle.log_response(img, taps)
        for k in range(0, taps.shape[0] // 2):
            assert Fraction(L[5, c - 1 - k]) == (b - a) * T[k + 1]
            assert Fraction(L[5, c + k]) == -(b - a) * T[k + 1]
        Z = oracle.zero_cross(L)
        z0 = (b - a) * (T[1] + max(T[1], T[2]))
        assert np.array_equal(np.nonzero(Z.any(axis=0))[0], [c])
        assert all(Fraction(v) == z0 for v in Z[:, c])
        sg = oracle.global_std(Z)
        assert sg == pytest.approx(math.sqrt(H * float(z0) ** 2 * (1 - 1 / W) / (H * W - 1)), rel=1e-13)
        S3 = oracle.local_std(Z, 3)
        assert np.allclose(S3[:, c - 1:c + 2], float(z0) / 2, rtol=1e-14)
        assert not S3[:, :c - 1].any() and not S3[:, c + 2:].any()
    out = oracle.extract(img, t1, t2, smooth=True, want_intermediates=True)
    expect = np.zeros((H, W), np.uint8)
    expect[:, c - 1:c + 2] = 1
    assert np.array_equal(out["E"], expect)
    assert np.array_equal(out["F"], expect)


def test_constant_image_gives_nothing():
    t1, t2 = _masks()
    for v in (0, 77, 255):
        out = oracle.extract(np.full((40, 33), v, np.uint8), t1, t2, want_intermediates=True)
        assert not out["F"].any() and not out["Z1"].any() and not out["Z2"].any()
        assert list(out["stats"]) == [0, 0, 0, 0]


# ---------------------------------------------------------------- eq. (2)
def test_global_std_matches_numpy():
    rng = np.random.default_rng(5)
    for n in (2, 3, 1000, 100003):
        z = rng.exponential(3.0, n) * (rng.random(n) < 0.4)
        assert oracle.global_std(z) == pytest.approx(np.std(z, ddof=1), rel=1e-12)
    assert oracle.global_std(np.array([5.0])) == 0.0


@pytest.mark.parametrize("win", [3, 5])
def test_local_std_matches_numpy_windows(win):
    rng = np.random.default_rng(9)
    Z = rng.exponential(2.0, (23, 19)) * (rng.random((23, 19)) < 0.5)
    r = win // 2
    P = np.pad(Z, r, mode="edge")
    ref = sliding_window_view(P, (win, win)).reshape(23, 19, -1).std(axis=-1, ddof=1)
    assert np.allclose(oracle.local_std(Z, win), ref, rtol=1e-12, atol=1e-300)


# ---------------------------------------------------------------- hybrid median (Sec. 3.4)
@pytest.mark.parametrize("win", [3, 5])
def test_hybrid_median_matches_numpy_median(win):
    rng = np.random.default_rng(13)
    E = rng.integers(0, 256, size=(21, 26)).astype(np.uint8)
    r = win // 2
    P = np.pad(E, r, mode="edge")
    Wv = sliding_window_view(P, (win, win))
    idx = np.arange(win)
    plus = np.concatenate([Wv[:, :, r, :], np.delete(Wv[:, :, :, r], r, axis=2)], axis=2)
    cross = np.concatenate([Wv[:, :, idx, idx], np.delete(Wv[:, :, idx, idx[::-1]], r, axis=2)], axis=2)
    ref = np.median(np.stack([np.median(plus, axis=2), np.median(cross, axis=2),
                              E.astype(np.float64)], axis=2), axis=2).astype(np.uint8)
    assert np.array_equal(oracle.hybrid_median(E, win), ref)


def test_hybrid_median_keeps_thin_lines_plain_median_erases_them():
    """Sec. 2 / Sec. 3.4: the plain median erases lines thinner than half the
    window; the hybrid median keeps them.  It still removes an isolated speck
    and fills an isolated hole."""
    E = np.zeros((30, 30), np.uint8)
    E[15, :] = 1                      # 1-px horizontal line
    E[:, 7] = 1                       # 1-px vertical line
    for i in range(30):               # 1-px diagonal
        E[i, i] = 1
    F = oracle.hybrid_median(E, 5)
    assert np.array_equal(F[2:-2, 2:-2], E[2:-2, 2:-2])
    assert not ndi.median_filter(E, size=5, mode="nearest")[15, 12:18].any()
    speck = np.zeros((9, 9), np.uint8)
    speck[4, 4] = 1
    assert not oracle.hybrid_median(speck, 5).any()
    hole = np.ones((9, 9), np.uint8)
    hole[4, 4] = 0
    assert oracle.hybrid_median(hole, 5).all()


# ---------------------------------------------------------------- whole pipeline vs brute force
def _exact_band(ex, key_v, key_t, tol=1e-9):
    """Pixels whose exact 3x3 variance is within tol (relative) of T^2."""
    V, T2 = ex[key_v], ex[key_t]
    H, W = len(V), len(V[0])
    out = np.zeros((H, W), bool)
    for y in range(H):
        for x in range(W):
            if abs(V[y][x] - T2) <= Fraction(tol) * max(T2, Fraction(1, 10 ** 30)):
                out[y, x] = True
    return out


@pytest.mark.parametrize("shape", [(1, 1), (1, 7), (6, 1), (2, 2), (5, 7), (9, 12), (13, 11)])
@pytest.mark.parametrize("masks", [((3, 0.5), (5, 0.8)), ((5, 0.8), (9, 1.4))])
def test_pipeline_matches_exact_brute_force(shape, masks):
    (s1, g1), (s2, g2) = masks
    t1 = oracle.log_mask(s1, g1, 16)[0]
    t2 = oracle.log_mask(s2, g2, 16)[0]
    rng = np.random.default_rng(hash(shape) % 1000)
    for trial in range(2):
        img = rng.integers(0, 256, size=shape).astype(np.uint8)
        if trial == 1:  # blocky image: many exact ties and zero responses
            img = (rng.integers(0, 2, size=shape) * 100).astype(np.uint8)
        for smooth, ms in ((True, 5), (False, 5), (True, 3)):
            o = oracle.extract(img, t1, t2, smooth=smooth, median_size=ms, want_intermediates=True)
            b = brute.extract(img.tolist(), t1.tolist(), t2.tolist(), smooth=smooth, median_size=ms)
            for j in (1, 2):
                assert [[Fraction(v) for v in row] for row in o[f"L{j}"].tolist()] == b[f"L{j}"]
                assert [[Fraction(v) for v in row] for row in o[f"Z{j}"].tolist()] == b[f"Z{j}"]
            band = _exact_band(b, "V1", "T2_1") | _exact_band(b, "V2", "T2_2")
            E_b = np.array(b["E"], np.uint8)
            assert np.array_equal(o["E"][~band], E_b[~band])
            if not band.any():
                assert np.array_equal(o["F"], np.array(b["F"], np.uint8))


def test_abs_mode_and_5x5_stage_match_brute_force():
    t1 = oracle.log_mask(3, 0.5, 16)[0]
    t2 = oracle.log_mask(5, 0.8, 16)[0]
    rng = np.random.default_rng(21)
    img = rng.integers(0, 256, size=(10, 11)).astype(np.uint8)
    for kw in (dict(std_mode=1, std_k=20.0), dict(std5_max=15.0), dict(zc_thresh=30.0)):
        o = oracle.extract(img, t1, t2, want_intermediates=True, **kw)
        b = brute.extract(img.tolist(), t1.tolist(), t2.tolist(), **kw)
        assert np.array_equal(o["E"], np.array(b["E"], np.uint8)), kw
        assert np.array_equal(o["F"], np.array(b["F"], np.uint8)), kw


def test_threads_do_not_change_results():
    img = scenes.config1(seed=4)[:200, :180]
    t1, t2 = _masks()
    a = oracle.extract(img, t1, t2, nthreads=1, want_intermediates=True)
    b = oracle.extract(img, t1, t2, nthreads=7, want_intermediates=True)
    for k in ("F", "E", "L1", "L2", "Z1", "Z2", "S1", "S2", "stats"):
        assert np.array_equal(a[k], b[k]), k


def test_config1_densities_are_plausible():
    """Not a paper value (the paper prints none): a sanity band on the
    synthetic 512^2 scene so that a gross regression shows up."""
    img = scenes.config1()
    t1, t2 = _masks()
    o = oracle.extract(img, t1, t2, want_intermediates=True)
    assert 0.45 < (o["Z1"] > 0).mean() < 0.7
    assert 0.25 < (o["Z2"] > 0).mean() < 0.45
    assert 0.02 < o["F"].mean() < 0.12


def test_masks_match_frozen_golden():
    """tests/golden/masks.json was written by tests/golden/make_golden.py
    (oracle only); a change to the mask construction must be deliberate."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "masks.json")) as f:
        gold = json.load(f)["masks"]
    for m in gold:
        taps, u = oracle.log_mask(m["size"], m["sigma"], m["grid_bits"])
        assert u == m["unit"]
        assert np.array_equal(np.round(taps.astype(np.float64) / u).astype(int), np.array(m["k"]))
