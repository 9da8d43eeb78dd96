"""GPU parity: liblogfx (through its C ABI) against the CPU oracle on the same
seeded inputs.  LoG responses and crossing strengths must agree bit for bit
(both are exact sums); extracted and output maps must agree except where
the oracle's deviation lies within 1e-5 of its threshold (band pixels), and
such mismatches must stay below 1e-6 of the pixels."""
import os

import numpy as np
import pytest

import oracle
from paper_1304_3992_amd import logfx, scenes
from parity import compare, masks, run_gpu, run_oracle, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    c = logfx.Context(0)
    yield c
    c.close()


def _rand(shape, maxv, seed, dtype):
    return np.random.default_rng(seed).integers(0, maxv + 1, size=shape).astype(dtype)


def _scene_crop(h, w, seed=1, bits=8):
    if bits == 8:
        return scenes.panchromatic(h, w, seed, n_rect=max(1, h * w // 6000), noise_sigma=4.0)
    return scenes.panchromatic(h, w, seed, n_rect=max(1, h * w // 3000), n_poly=3,
                               noise_sigma=12.0, sp_density=0.05, bits=bits)


def _zero_pixel_steps():
    """Noise-free three-level steps, 0 | 50 | 100 across plus 0 | 40 | 80
    down: the middle column and row are centres of antisymmetry, so with
    zero-sum masks the LoG is exactly 0 on them (away from where they
    cross) between neighbours of opposite signs -- the crossing rule's
    zero-pixel case, left / right and up / down -- beside flat areas of
    exact zeros."""
    a = np.zeros(300, np.int32)
    a[101] = 50
    a[102:] = 100
    b = np.zeros(150, np.int32)
    b[70] = 40
    b[71:] = 80
    img = b[:, None] + a[None, :]
    img[20:40, 200:230] += 30
    return img.astype(np.uint8)


MAP_CASES = [
    # (name, image factory, bits, mask pair, grid bits)
    ("zero_pixel_rule", _zero_pixel_steps, 0, ((5, 0.8), (9, 1.4)), 16),
    ("zero_pixel_rule_r1r3", _zero_pixel_steps, 0, ((3, 0.5), (7, 1.0)), 16),
    ("c1crop_u8", lambda: scenes.config1()[:300, :250], 0, ((5, 0.8), (9, 1.4)), 16),
    ("rand_u8_ragged", lambda: _rand((131, 301), 255, 3, np.uint8), 0, ((5, 0.8), (9, 1.4)), 16),
    ("scene_u11", lambda: _scene_crop(200, 333, 5, 11), 11, ((5, 0.8), (9, 1.4)), 16),
    ("r1r2_u12", lambda: _rand((90, 260), 4095, 20, np.uint16), 12, ((3, 0.5), (5, 0.8)), 16),
    ("r2r3_u12", lambda: _rand((75, 140), 4095, 21, np.uint16), 12, ((5, 0.8), (7, 1.0)), 16),
    ("rand_u16_fp64", lambda: _rand((97, 150), 65535, 4, np.uint16), 16, ((5, 0.8), (9, 1.4)), 16),
    ("grid23_fp64", lambda: scenes.config1()[:128, :300], 0, ((5, 0.8), (9, 1.4)), 23),
    ("swapped_sizes", lambda: _rand((70, 90), 255, 6, np.uint8), 0, ((9, 1.4), (3, 0.5)), 16),
    ("r1r1", lambda: _rand((65, 129), 255, 7, np.uint8), 0, ((3, 0.5), (3, 0.9)), 16),
    ("r3r3", lambda: _rand((40, 200), 255, 8, np.uint8), 0, ((7, 1.0), (7, 1.2)), 16),
    ("r4r4_fp64", lambda: _rand((50, 77), 65535, 9, np.uint16), 16, ((9, 1.4), (9, 2.0)), 16),
    ("one_pixel", lambda: np.array([[77]], np.uint8), 0, ((5, 0.8), (9, 1.4)), 16),
    ("one_row", lambda: _rand((1, 200), 255, 10, np.uint8), 0, ((5, 0.8), (9, 1.4)), 16),
    ("one_col", lambda: _rand((150, 1), 255, 11, np.uint8), 0, ((5, 0.8), (9, 1.4)), 16),
]


@pytest.mark.parametrize("name,make,bits,pair,gb", MAP_CASES, ids=[c[0] for c in MAP_CASES])
def test_maps_bit_exact(ctx, name, make, bits, pair, gb):
    import torch
    img = make()
    orc_t, lib_t = masks(pair, gb)
    o = run_oracle(img, orc_t)
    maps = ctx.extract_maps(to_device(img), logfx.Params(*lib_t), bits=bits)
    torch.cuda.synchronize()
    for k in ("L1", "L2", "Z1", "Z2"):
        g = maps[k].cpu().numpy()
        ref = o[k]
        # the 1e-5 relative bound holds trivially; exact equality is the real bar
        assert np.array_equal(g, ref), (k, int((g != ref).sum()))


PACKED_CASES = [
    # (name, image factory, bits, mask pair, grid bits, packed form applies)
    ("u8_r2r4", lambda: _rand((131, 301), 255, 40, np.uint8), 0, ((5, 0.8), (9, 1.4)), 16, True),
    ("u11_r2r4", lambda: _scene_crop(200, 333, 41, 11), 11, ((5, 0.8), (9, 1.4)), 16, True),
    ("u13_r1r2", lambda: _rand((90, 260), 8191, 42, np.uint16), 13, ((3, 0.5), (5, 0.8)), 14, True),
    # 13-bit extremes: sums of four pixels reach 4 * 8191, the top of int16
    ("u13_extremes", lambda: ((np.indices((96, 200)).sum(0) // 3 % 2) * 8191 +
                              (_rand((96, 200), 1, 48, np.uint16) * 8191)).clip(0, 8191).astype(np.uint16),
     13, ((5, 0.8), (9, 1.4)), 13, True),
    ("u12_r3r3", lambda: _rand((75, 140), 4095, 43, np.uint16), 12, ((7, 1.0), (7, 1.2)), 15, True),
    ("u12_r4r4_wide", lambda: _rand((60, 500), 4095, 44, np.uint16), 12, ((9, 1.4), (9, 2.0)), 12, True),
    ("u8_r1r1", lambda: _rand((65, 129), 255, 45, np.uint8), 0, ((3, 0.5), (3, 0.9)), 16, True),
    ("zero_pixel_rule", _zero_pixel_steps, 0, ((5, 0.8), (9, 1.4)), 16, True),
    # 14-bit pixels on a 12-bit tap grid: exact in int32, but four pixels
    # overflow int16, so the 32-bit form runs whatever the option says
    ("u14_grid12_r2r4", lambda: _rand((70, 300), 16383, 46, np.uint16), 14, ((5, 0.8), (9, 1.4)), 12, False),
]


@pytest.mark.parametrize("name,make,bits,pair,gb,packed", PACKED_CASES, ids=[c[0] for c in PACKED_CASES])
def test_packed_and_32bit_forms_agree(ctx, name, make, bits, pair, gb, packed):
    """The integer path with the LoG on packed 16-bit sums (the default where
    pixels and taps fit) and in the 32-bit form: L and Z bit-identical to each
    other and to the oracle, and the same output map."""
    import torch
    img = make()
    orc_t, lib_t = masks(pair, gb)
    params = logfx.Params(*lib_t)
    dev = to_device(img)
    assert logfx.check_params(logfx.image(dev, bits), params) == logfx.PATH_INT32
    o = run_oracle(img, orc_t)
    got = {}
    try:
        for form in (1, 0):
            ctx.set_option(logfx.OPT_PACKED_LOG, form)
            maps = ctx.extract_maps(dev, params, bits=bits)
            out = ctx.extract(dev, params, bits=bits)
            torch.cuda.synchronize()
            got[form] = ({k: maps[k].cpu().numpy() for k in ("L1", "L2", "Z1", "Z2")}, out.cpu().numpy())
    finally:
        ctx.set_option(logfx.OPT_PACKED_LOG, 1)
    for k in ("L1", "L2", "Z1", "Z2"):
        assert np.array_equal(got[1][0][k], o[k]), (k, int((got[1][0][k] != o[k]).sum()))
        assert np.array_equal(got[0][0][k], got[1][0][k]), k
    assert np.array_equal(got[0][1], got[1][1])
    compare(got[1][1], o, smooth=True)


def _edge_mask(edge, corner, centre=-65534.0):
    """A 3x3 D4-symmetric integer mask: centre, 4-neighbour taps, corners."""
    m = np.full((3, 3), corner, np.float32)
    m[0, 1] = m[1, 0] = m[1, 2] = m[2, 1] = edge
    m[1, 1] = centre
    return m


@pytest.mark.parametrize("edge,corner", [(32767.0, -32768.0), (32769.0, -32768.0)],
                         ids=["int16_limits_packed", "past_int16_32bit"])
def test_packed_form_at_the_int16_tap_limit(ctx, edge, corner):
    """Taps at the ends of int16 (packed form, the centre tap in the 24-bit
    multiply) and just past them (the 32-bit form; an odd tap keeps the grid
    unit at 1, where an even one would halve every tap), on 11-bit pixels
    with blocks at 0 and 2047 so that the row-pair sums reach four times the
    maximum: L and Z bit-identical to the oracle in both forms (which form
    runs: test_packed_form_selection_logged)."""
    import torch
    rng = np.random.default_rng(49)
    img = rng.integers(0, 2048, (80, 300)).astype(np.uint16)
    img[10:30, 20:120] = 2047
    img[40:60, 150:260] = 0
    img[30:40, :] = (np.indices((10, 300)).sum(0) % 2 * 2047).astype(np.uint16)
    m1 = _edge_mask(edge, corner)
    m2 = logfx.make_log_mask(9, 1.4, 16)[0]
    o = oracle.extract(img, m1.astype(np.float64), oracle.log_mask(9, 1.4, 16)[0], want_intermediates=True)
    params = logfx.Params(m1, m2)
    dev = to_device(img)
    assert logfx.check_params(logfx.image(dev, 11), params) == logfx.PATH_INT32
    maps = ctx.extract_maps(dev, params, bits=11)
    torch.cuda.synchronize()
    for k in ("L1", "L2", "Z1", "Z2"):
        g = maps[k].cpu().numpy()
        assert np.array_equal(g, o[k]), (k, int((g != o[k]).sum()))


SELECTION_SCRIPT = r"""
import sys
sys.path.insert(0, %r)
sys.path.insert(0, %r)
import numpy as np, torch
from paper_1304_3992_amd import logfx
from parity import masks, to_device
ctx = logfx.Context(0)
rng = np.random.default_rng(47)
def edge(e):
    m = np.full((3, 3), -32768.0, np.float32)
    m[0, 1] = m[1, 0] = m[1, 2] = m[2, 1] = e
    m[1, 1] = -65534.0
    return m
cases = [(rng.integers(0, 2048, (40, 70)).astype(np.uint16), 11, masks(grid_bits=16)[1], 1),
         (rng.integers(0, 2048, (41, 70)).astype(np.uint16), 11, masks(grid_bits=16)[1], 0),
         (rng.integers(0, 16384, (42, 70)).astype(np.uint16), 14, masks(grid_bits=12)[1], 1),
         (rng.integers(0, 2048, (43, 70)).astype(np.uint16), 11, (edge(32767.0), masks()[1][1]), 1),
         (rng.integers(0, 2048, (44, 70)).astype(np.uint16), 11, (edge(32769.0), masks()[1][1]), 1)]
for img, bits, taps, form in cases:
    ctx.set_option(logfx.OPT_PACKED_LOG, form)
    ctx.extract(to_device(img), logfx.Params(*taps), bits=bits)
    torch.cuda.synchronize()
print("done")
"""


def test_packed_form_selection_logged():
    """Which form runs, as the call log states it (a child process: the
    log setting is read once): packed for 11-bit pixels, the 32-bit form
    when the option turns it off, for 14-bit pixels whatever the option
    says, and at the int16 limit of the non-centre taps."""
    import subprocess
    import sys
    here = os.path.dirname(os.path.abspath(__file__))
    env = dict(os.environ, LOGFX_LOG="1")
    r = subprocess.run([sys.executable, "-c", SELECTION_SCRIPT % (os.path.dirname(here), here)], env=env,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "done" in r.stdout, r.stderr[-2000:]
    lines = [ln for ln in r.stderr.splitlines() if ln.startswith("[liblogfx] extract:")]
    assert len(lines) == 5, r.stderr[-2000:]
    assert "40 x 70, int32 (packed) path" in lines[0]
    assert "41 x 70, int32 path" in lines[1]
    assert "42 x 70, int32 path" in lines[2]
    assert "43 x 70, int32 (packed) path" in lines[3]   # non-centre taps 32767 and -32768
    assert "44 x 70, int32 path" in lines[4]            # one at 32769


EXTRACT_CASES = [
    ("c1", lambda: scenes.config1(), 0, {}),
    ("c1_nosmooth", lambda: scenes.config1(), 0, dict(smooth=False)),
    ("c1_med3", lambda: scenes.config1(), 0, dict(median_size=3)),
    ("c1_abs", lambda: scenes.config1(), 0, dict(std_mode=logfx.STD_ABS, std_k=6.0)),
    ("c1_zcthr", lambda: scenes.config1(), 0, dict(zc_thresh=2.0)),
    ("ragged_u8", lambda: _scene_crop(700, 333, 12), 0, {}),
    ("ragged_u11", lambda: _scene_crop(257, 449, 13, 11), 11, {}),
    ("u16_fp64", lambda: _scene_crop(190, 230, 14, 16), 16, {}),
    ("tiny_2x2", lambda: _rand((2, 2), 255, 15, np.uint8), 0, {}),
    ("tiny_1x1", lambda: np.array([[9]], np.uint8), 0, {}),
    ("row_1x300", lambda: _rand((1, 300), 255, 16, np.uint8), 0, {}),
    ("col_300x1", lambda: _rand((300, 1), 255, 17, np.uint8), 0, {}),
    ("thin_3x500", lambda: _rand((3, 500), 255, 18, np.uint8), 0, dict(median_size=3)),
    ("checker", lambda: (np.indices((64, 96)).sum(0) % 2 * 200).astype(np.uint8), 0, {}),
    ("saturated", lambda: (np.random.default_rng(19).random((120, 140)) < 0.5).astype(np.uint16)
     * 65535, 16, {}),
    ("constant", lambda: np.full((100, 100), 33, np.uint8), 0, {}),
    ("wide_9x180000", lambda: _rand((9, 180000), 255, 22, np.uint8), 0, {}),
    ("tall_180000x9", lambda: _rand((180000, 9), 255, 23, np.uint8), 0, {}),
    ("wide_u11_5x70001", lambda: _scene_crop(5, 70001, 24, 11), 11, dict(median_size=3)),
]


@pytest.mark.parametrize("rows1,rows2", [(40, 24), (64, 64), (48, 96), (64, 128)])
@pytest.mark.parametrize("std5", [False, True])
def test_strip_heights(ctx, rows1, rows2, std5):
    """Other strip heights than the tuned ones, on a ragged 11-bit crop
    whose last strips are short: pass 1's rows read a step ahead and pass
    2's rows shared with the strip below, read first, at every position of
    a strip, with the 5x5 first stage and without."""
    img = _scene_crop(349, 301, 25, 11)
    orc_t, lib_t = masks()
    kw = dict(std5_max=_std5_threshold(img, orc_t, 0.5)[0]) if std5 else {}
    o = run_oracle(img, orc_t, **kw)
    opts = (logfx.OPT_ROWS1, logfx.OPT_ROWS2)
    saved = [ctx.get_option(k) for k in opts]
    try:
        ctx.set_option(logfx.OPT_ROWS1, rows1)
        ctx.set_option(logfx.OPT_ROWS2, rows2)
        F, rep = run_gpu(ctx, img, lib_t, bits=11, **kw)
    finally:
        for k, v in zip(opts, saved):
            ctx.set_option(k, v)
    compare(F, o, smooth=True, **kw)


@pytest.mark.parametrize("name,make,bits,kw", EXTRACT_CASES, ids=[c[0] for c in EXTRACT_CASES])
def test_extract_parity(ctx, name, make, bits, kw):
    img = make()
    orc_t, lib_t = masks()
    o = run_oracle(img, orc_t, **kw)
    F, rep = run_gpu(ctx, img, lib_t, bits=bits, **kw)
    compare(F, o, smooth=kw.get("smooth", True), median_size=kw.get("median_size", 5))
    # the report: exact counts and the global statistics of eq. (2)
    assert rep["pixels"] == img.size
    assert rep["zc_count"] == [int((o["Z1"] != 0).sum()), int((o["Z2"] != 0).sum())]
    assert rep["output"] == int(F.sum())
    np.testing.assert_allclose(rep["sigma_g"], o["stats"][:2], rtol=1e-12, atol=0)
    np.testing.assert_allclose(rep["thresh"], o["stats"][2:], rtol=1e-12, atol=0)
    if name == "constant":
        assert not F.any() and rep["sigma_g"] == [0.0, 0.0]


def test_step_edge_band(ctx):
    """Worked example: a vertical step gives exactly the three columns around
    it (see the oracle pins); the GPU must reproduce it."""
    H, W, c = 32, 64, 20
    img = np.full((H, W), 40, np.uint8)
    img[:, c:] = 200
    _, lib_t = masks()
    F, _ = run_gpu(ctx, img, lib_t)
    expect = np.zeros((H, W), np.uint8)
    expect[:, c - 1:c + 2] = 1
    assert np.array_equal(F, expect)


def test_pitch_larger_than_width(ctx):
    img = _scene_crop(150, 210, 20)
    orc_t, lib_t = masks()
    o = run_oracle(img, orc_t)
    F, _ = run_gpu(ctx, img, lib_t, pitch=333)
    compare(F, o, smooth=True)


@pytest.mark.parametrize("dtype,bits,off,pitch", [(np.uint8, 0, 3, 1001), (np.uint16, 11, 5, 517),
                                                  (np.uint8, 0, 1, 777), (np.uint16, 11, 1, 1203)])
def test_unaligned_base_and_pitch(ctx, dtype, bits, off, pitch):
    """Images whose first pixel and row pitch are at odd element offsets in
    their buffer (interior chunks are read by unaligned vector loads): the
    map equals the same image's map from a contiguous aligned buffer bit for
    bit, and the oracle's under the band rule.  Widths span several tiles
    and a ragged tail."""
    import torch
    img = _scene_crop(230, pitch - 13, 25 + off, 11 if bits else 8).astype(dtype)
    H, W = img.shape
    orc_t, lib_t = masks()
    a = img.view(np.int16) if dtype == np.uint16 else img
    buf = torch.zeros(off + H * pitch, dtype=torch.from_numpy(a[:1, :1].copy()).dtype)
    flat = torch.from_numpy(np.ascontiguousarray(a))
    for y in range(H):
        buf[off + y * pitch: off + y * pitch + W] = flat[y]
    dev = buf.cuda().as_strided((H, W), (pitch, 1), off)
    params = logfx.Params(*lib_t)
    F = ctx.extract(dev, params, bits=bits)
    ref = ctx.extract(to_device(img), params, bits=bits)
    torch.cuda.synchronize()
    assert torch.equal(F, ref)
    compare(F.cpu().numpy(), run_oracle(img, orc_t), smooth=True)


def test_repeatable_and_tile_independent(ctx):
    """Two runs give identical bytes, and so does a context with another tile
    shape (tiles change the reduction order of the global sums only)."""
    img = _scene_crop(600, 500, 21)
    _, lib_t = masks()
    a, ra = run_gpu(ctx, img, lib_t)
    b, rb = run_gpu(ctx, img, lib_t)
    assert np.array_equal(a, b) and ra == rb
    old = os.environ.get("LOGFX_TILE")
    os.environ["LOGFX_TILE"] = "24,40"
    try:
        c2 = logfx.Context(0)
    finally:
        if old is None:
            del os.environ["LOGFX_TILE"]
        else:
            os.environ["LOGFX_TILE"] = old
    c, rc = run_gpu(c2, img, lib_t)
    c2.close()
    assert np.array_equal(a, c)
    assert rc["zc_count"] == ra["zc_count"] and rc["output"] == ra["output"]


def test_side_stream(ctx):
    import torch
    img = scenes.config1(seed=22)
    orc_t, lib_t = masks()
    o = run_oracle(img, orc_t)
    s = torch.cuda.Stream()
    t = to_device(img)
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        out = ctx.extract(t, logfx.Params(*lib_t), stream=s)
    s.synchronize()
    compare(out.cpu().numpy(), o, smooth=True)


def test_config2_full_size(ctx):
    """8192^2 11-bit scene with 20000 rectangles, 500 polylines, noise sigma
    12 and 5 % impulses, at the launch configuration the benchmark uses: the
    whole output map against the oracle, and the LoG / strength maps on a
    band of rows."""
    import torch
    img = scenes.config2()
    orc_t, lib_t = masks()
    o = run_oracle(img, orc_t)
    F, rep = run_gpu(ctx, img, lib_t, bits=11)
    info = compare(F, o, smooth=True)
    assert rep["path"] == logfx.PATH_INT32
    np.testing.assert_allclose(rep["sigma_g"], o["stats"][:2], rtol=1e-12)
    # the benchmark's own launch: strip heights chosen by the tuner
    opts = (logfx.OPT_ROWS1, logfx.OPT_ROWS2, logfx.OPT_PERSISTENT)
    saved = [ctx.get_option(k) for k in opts]
    try:
        ctx.tune(to_device(img), logfx.Params(*lib_t), bits=11, reps=3)
        Ft, _ = run_gpu(ctx, img, lib_t, bits=11)
        tuned = [ctx.get_option(k) for k in opts]
    finally:
        for k, v in zip(opts, saved):
            ctx.set_option(k, v)
    assert np.array_equal(Ft, F), tuned
    maps = ctx.extract_maps(to_device(img), logfx.Params(*lib_t), bits=11)
    torch.cuda.synchronize()
    for k in ("L1", "L2", "Z1", "Z2"):
        g = maps[k]
        for r0 in (0, 4093, 8192 - 70):
            assert np.array_equal(g[r0:r0 + 70].cpu().numpy(), o[k][r0:r0 + 70]), (k, r0)
    del maps
    print("config2", info)


@pytest.mark.parametrize("kind", ["grid23_crop", "u16_pixels"])
def test_fp64_path_large(ctx, kind):
    """The FP64 path at 4096^2: a crop of the 8192^2 scene with masks on the
    23-bit grid (the finest an FP32 tap holds; its sums exceed the int32
    bound), or 16-bit pixels with the default masks.  The whole output map
    against the oracle with the band rule, and the LoG and strength maps bit
    for bit on bands of rows at the top, middle and bottom."""
    import torch
    if kind == "grid23_crop":
        img, bits, gb = scenes.config2()[2048:6144, 1024:5120].copy(), 11, 23
    else:
        img = scenes.panchromatic(4096, 4096, 31, n_rect=5000, n_poly=120, noise_sigma=300.0,
                                  sp_density=0.02, bits=16)
        bits, gb = 16, 16
    orc_t, lib_t = masks(grid_bits=gb)
    o = run_oracle(img, orc_t)
    F, rep = run_gpu(ctx, img, lib_t, bits=bits)
    assert rep["path"] == logfx.PATH_FP64
    info = compare(F, o, smooth=True)
    np.testing.assert_allclose(rep["sigma_g"], o["stats"][:2], rtol=1e-12)
    maps = ctx.extract_maps(to_device(img), logfx.Params(*lib_t), bits=bits)
    torch.cuda.synchronize()
    for k in ("L1", "L2", "Z1", "Z2"):
        for r0 in (0, 2000, 4096 - 70):
            assert np.array_equal(maps[k][r0:r0 + 70].cpu().numpy(), o[k][r0:r0 + 70]), (k, r0)
    del maps
    torch.cuda.empty_cache()
    print(kind, info)


def test_largest_single_image_16400(ctx):
    """A 16400^2 image in one call: 269 Mpixel, 2.15 GB of stored strength
    pairs (byte offsets past 2^31), 67 x 257 pass-1 tiles; the whole output
    against the oracle with the band rule."""
    import torch
    img = _rand((16400, 16400), 2047, 25, np.uint16)
    orc_t, lib_t = masks()
    o = run_oracle(img, orc_t)
    F, rep = run_gpu(ctx, img, lib_t, bits=11)
    info = compare(F, o, smooth=True)
    assert rep["output"] == int(F.sum())
    np.testing.assert_allclose(rep["sigma_g"], o["stats"][:2], rtol=1e-12)
    del o, F
    torch.cuda.empty_cache()
    print("16384^2", info)


@pytest.mark.parametrize("name,make,bits,kw", [c for c in EXTRACT_CASES if c[0] in
                                               ("c1", "c1_nosmooth", "c1_med3", "ragged_u11", "u16_fp64",
                                                "tiny_1x1", "row_1x300", "col_300x1", "thin_3x500")],
                         ids=lambda v: v if isinstance(v, str) else "")
def test_stored_and_recomputed_strengths_agree(ctx, name, make, bits, kw):
    """Pass 2 on the strengths stored by pass 1 and pass 2 recomputing them
    from the image run the same FP64 operations: same bytes, same report."""
    img = make()
    _, lib_t = masks()
    ctx.set_option(logfx.OPT_STORE_Z, 0)
    try:
        a, ra = run_gpu(ctx, img, lib_t, bits=bits, **kw)
    finally:
        ctx.set_option(logfx.OPT_STORE_Z, 1)
    b, rb = run_gpu(ctx, img, lib_t, bits=bits, **kw)
    assert np.array_equal(a, b)
    assert ra == rb


def _std5_threshold(img, orc_t, q, **kw):
    """A 5x5-stage threshold at quantile q of the oracle's own 5x5
    deviations (the larger of the two masks') at the pixels it extracts
    without the stage, so that the stage removes part of E."""
    o = run_oracle(img, orc_t, **kw)
    s5 = np.maximum(oracle.local_std(o["Z1"], 5), oracle.local_std(o["Z2"], 5))
    vals = np.unique(s5[o["E"] > 0])
    if vals.size < 2:
        return 1.0, o
    # halfway between two neighbouring values: no pixel sits on the threshold
    k = min(int(q * (vals.size - 1)), vals.size - 2)
    return float(0.5 * (vals[k] + vals[k + 1])), o


STD5_CASES = [
    ("c1_q50", lambda: scenes.config1(), 0, 0.5, {}),
    ("c1_q80_med3", lambda: scenes.config1(), 0, 0.8, dict(median_size=3)),
    ("c1_zero", lambda: scenes.config1(), 0, None, {}),
    ("ragged_u11_q60", lambda: _scene_crop(257, 449, 13, 11), 11, 0.6, {}),
    ("ragged_u8_nosmooth", lambda: _scene_crop(700, 333, 12), 0, 0.4, dict(smooth=False)),
    ("abs_mode", lambda: scenes.config1(), 0, 0.5, dict(std_mode=logfx.STD_ABS, std_k=6.0)),
    ("tiny_2x2", lambda: _rand((2, 2), 255, 15, np.uint8), 0, 0.5, {}),
    ("row_1x300", lambda: _rand((1, 300), 255, 16, np.uint8), 0, 0.5, {}),
    ("col_300x1", lambda: _rand((300, 1), 255, 17, np.uint8), 0, 0.5, {}),
    ("u16_fp64", lambda: _scene_crop(190, 230, 14, 16), 16, 0.5, {}),
]


@pytest.mark.parametrize("name,make,bits,q,kw", STD5_CASES, ids=[c[0] for c in STD5_CASES])
def test_first_stage_5x5(ctx, name, make, bits, q, kw):
    """The paper's 5x5 first deviation stage (Sec. 4.1, read as: E_j also
    needs the 5x5 deviation of Z_j above std5_max) against the oracle, with
    the band rule extended to the 5x5 deviations."""
    img = make()
    orc_t, lib_t = masks()
    if q is None:
        t, o_off = 0.0, run_oracle(img, orc_t, **kw)
    else:
        t, o_off = _std5_threshold(img, orc_t, q, **kw)
    o = run_oracle(img, orc_t, std5_max=t, **kw)
    F, rep = run_gpu(ctx, img, lib_t, bits=bits, std5_max=t, **kw)
    info = compare(F, o, smooth=kw.get("smooth", True), median_size=kw.get("median_size", 5), std5_max=t)
    assert rep["output"] == int(F.sum())
    assert abs(rep["extracted"] - int(o["E"].sum())) <= info["band"]
    # the stage only removes pixels from E
    assert not (o["E"] & ~o_off["E"]).any()
    if q is not None and q >= 0.5 and img.size > 10000:
        assert o["E"].sum() < o_off["E"].sum()


def test_first_stage_5x5_batch_and_recompute_setting(ctx):
    """With the 5x5 stage a batch gives each tile its single-call output, and
    the stage runs on stored strengths even when the context is set to
    recompute them."""
    import torch
    tiles = scenes.config3(n=5, seed=77, base_seed=7700, lo=60, hi=700)
    orc_t, lib_t = masks()
    t, _ = _std5_threshold(tiles[0], orc_t, 0.5)
    params = logfx.Params(*lib_t, std5_max=t)
    devs = [to_device(x) for x in tiles]
    outs = [torch.empty(x.shape, dtype=torch.uint8, device="cuda") for x in tiles]
    ctx.extract_batch(devs, params, outs, bits=8)
    singles = []
    ctx.set_option(logfx.OPT_STORE_Z, 0)
    try:
        for d in devs:
            singles.append(ctx.extract(d, params, bits=8))
    finally:
        ctx.set_option(logfx.OPT_STORE_Z, 1)
    torch.cuda.synchronize()
    for i, (b, s) in enumerate(zip(outs, singles)):
        assert torch.equal(b, s), i
        o = run_oracle(tiles[i], orc_t, std5_max=t)
        compare(s.cpu().numpy(), o, smooth=True, std5_max=t)


def _midpoint(values, q):
    """Halfway between two neighbouring distinct values near quantile q."""
    v = np.unique(values)
    k = min(int(q * (v.size - 1)), v.size - 2)
    return float(0.5 * (v[k] + v[k + 1]))


@pytest.mark.parametrize("smooth", [True, False])
def test_paper_rule_and_masks(ctx, smooth):
    """The paper's own configuration (Sec. 4.1): two 5x5 masks of variance
    0.5 and 20, a zero-crossing threshold (Sec. 3.2), the 5x5 first stage
    and the 3x3 test with absolute thresholds.  Thresholds are taken halfway
    between neighbouring oracle values so that no pixel sits on one."""
    img = scenes.config1()
    orc_t, lib_t = masks(((5, 0.5 ** 0.5), (5, 20 ** 0.5)), 16)
    o0 = run_oracle(img, orc_t)
    z = np.concatenate([o0["Z1"][o0["Z1"] > 0], o0["Z2"][o0["Z2"] > 0]])
    zc = _midpoint(z, 0.3)
    o1 = run_oracle(img, orc_t, zc_thresh=zc)
    s3 = np.concatenate([o1["S1"][o1["S1"] > 0], o1["S2"][o1["S2"] > 0]])
    kw = dict(zc_thresh=zc, std_mode=logfx.STD_ABS, std_k=_midpoint(s3, 0.7))
    o2 = run_oracle(img, orc_t, **kw)
    s5 = np.maximum(oracle.local_std(o2["Z1"], 5), oracle.local_std(o2["Z2"], 5))
    kw["std5_max"] = _midpoint(s5[o2["E"] > 0], 0.4)
    o = run_oracle(img, orc_t, smooth=smooth, **kw)
    F, rep = run_gpu(ctx, img, lib_t, smooth=smooth, **kw)
    info = compare(F, o, smooth=smooth, std5_max=kw["std5_max"])
    assert rep["zc_count"] == [int((o["Z1"] != 0).sum()), int((o["Z2"] != 0).sum())]
    assert abs(rep["extracted"] - int(o["E"].sum())) <= info["band"]
    assert 0 < o["E"].sum() < o2["E"].sum()   # every stage is active


CASCADE_CASES = [
    ("c1_5_3", lambda: scenes.config1(), 0, dict(median_cascade=(3,))),
    ("c1_5_3_5", lambda: scenes.config1(), 0, dict(median_cascade=(3, 5))),
    ("c1_3_5_3_5", lambda: scenes.config1(), 0, dict(median_size=3, median_cascade=(5, 3, 5))),
    ("ragged_u11_5_3", lambda: _scene_crop(257, 449, 13, 11), 11, dict(median_cascade=(3,))),
    ("ragged_u8_5_5", lambda: _scene_crop(700, 333, 12), 0, dict(median_cascade=(5,))),
    ("tiny_2x2", lambda: _rand((2, 2), 255, 15, np.uint8), 0, dict(median_cascade=(5, 3))),
    ("row_1x300", lambda: _rand((1, 300), 255, 16, np.uint8), 0, dict(median_cascade=(3,))),
    ("col_300x1", lambda: _rand((300, 1), 255, 17, np.uint8), 0, dict(median_cascade=(5, 3))),
    ("nosmooth_ignored", lambda: scenes.config1(), 0, dict(smooth=False, median_cascade=(3, 5))),
]


@pytest.mark.parametrize("name,make,bits,kw", CASCADE_CASES, ids=[c[0] for c in CASCADE_CASES])
def test_median_cascade(ctx, name, make, bits, kw):
    """Further hybrid median levels (Sec. 3.4 / Sec. 4.2): the output equals
    the oracle's single-level output filtered again by the oracle's hybrid
    median with each further window, level by level; band pixels excuse
    mismatches within the summed radius of all levels."""
    img = make()
    orc_t, lib_t = masks()
    cas = kw.pop("median_cascade")
    smooth = kw.get("smooth", True)
    o = run_oracle(img, orc_t, **kw)
    ref = o["F"]
    radius = kw.get("median_size", 5) // 2 if smooth else 0
    if smooth:
        for m in cas:
            ref = oracle.hybrid_median(ref, m)
            radius += m // 2
    F, rep = run_gpu(ctx, img, lib_t, bits=bits, median_cascade=cas, **kw)
    compare(F, dict(o, F=ref), smooth=smooth, radius=radius)
    assert rep["output"] == int(F.sum())


def test_median_cascade_batch_equals_singles(ctx):
    """A batch with two further levels gives each tile its single-call
    output (the levels ping-pong between the outputs and the context's
    scratch map, image by image)."""
    import torch
    tiles = scenes.config3(n=6, seed=79, base_seed=7900, lo=60, hi=600)
    _, lib_t = masks()
    for cas in ((3,), (3, 5)):
        params = logfx.Params(*lib_t, median_cascade=cas)
        devs = [to_device(x) for x in tiles]
        outs, reps = ctx.extract_batch(devs, params, bits=8, report=True)
        for i, d in enumerate(devs):
            s, r = ctx.extract(d, params, bits=8, report=True)
            torch.cuda.synchronize()
            assert torch.equal(outs[i], s), (cas, i)
            assert reps[i]["output"] == r["output"] == int(s.sum().item())


def _rounding_cone(o, scales, n_terms):
    """Pixels whose output may legitimately differ when both sides round
    their FP64 LoG sums (LOGFX_ALLOW_INEXACT).  Each side's sum of n_terms
    products errs by at most n_terms * 2^-53 * sum|m||x| (the standard
    bound for recursive summation), so the two responses differ by at most
    twice that, delta.  A crossing decision (Sec. 3.2) can flip only where a
    response lies within delta of zero, or where the magnitudes of two
    opposite-sign neighbours lie within the sum of their deltas of each
    other.  Such a decision reaches E through the 3x3 deviation (radius 1);
    a deviation within the relative band of its threshold decides E
    directly; the median spreads E's doubt by its own radius."""
    from parity import band, dilate
    unsure = np.zeros(o["F"].shape, bool)
    for L, sc in ((o["L1"], scales[0]), (o["L2"], scales[1])):
        d = 2.0 * n_terms * 2.0 ** -53 * sc
        unsure |= np.abs(L) <= d
        Lp, dp = np.pad(L, 1, mode="edge"), np.pad(d, 1, mode="edge")
        H, W = L.shape
        for dy, dx in ((-1, 0), (1, 0), (0, -1), (0, 1)):
            q = Lp[1 + dy:1 + dy + H, 1 + dx:1 + dx + W]
            dq = dp[1 + dy:1 + dy + H, 1 + dx:1 + dx + W]
            maybe_opposite = (L * q < 0) | (np.abs(q) <= dq)
            unsure |= maybe_opposite & (np.abs(np.abs(L) - np.abs(q)) <= d + dq)
    return dilate(dilate(unsure, 1) | band(o), 2)


def test_allow_inexact_masks(ctx):
    """With LOGFX_ALLOW_INEXACT a mask pair of very wide dynamic range runs
    on the FP64 path: the LoG responses agree with the oracle's within
    1e-5 of sum |m| |x| (the oracle's FP64 sums round too), the report says
    the sums were rounded, and every output pixel that differs from the
    oracle's lies in the cone of a decision that the summation bound leaves
    open (_rounding_cone)."""
    import torch
    from test_abi import _wide_range_masks
    img = scenes.config1()
    m1, m2 = _wide_range_masks()
    params = logfx.Params(m1, m2, flags=logfx.ALLOW_INEXACT)
    maps = ctx.extract_maps(to_device(img), params)
    F, rep = run_gpu(ctx, img, (m1, m2), flags=logfx.ALLOW_INEXACT)
    torch.cuda.synchronize()
    assert rep["inexact"] == 1 and rep["path"] == logfx.PATH_FP64
    scales = []
    for k, m in (("L1", m1), ("L2", m2)):
        ref = oracle.log_response(img, m)
        scale = oracle.log_response(img, np.abs(m))   # sum |m| |x| (pixels are >= 0)
        scales.append(scale)
        assert np.all(np.abs(maps[k].cpu().numpy() - ref) <= 1e-5 * scale), k
    o = run_oracle(img, (m1, m2))
    cone = _rounding_cone(o, scales, n_terms=81)
    mism = F != o["F"]
    assert not (mism & ~cone).any(), int((mism & ~cone).sum())
    print("inexact masks:", int(mism.sum()), "differing pixels,", int(cone.sum()), "in the rounding cone")
