"""Host-side checks of liblogfx (no GPU): the library loads, exports every
symbol include/logfx.h declares, builds the same masks as the oracle, and
rejects invalid requests before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_1304_3992_amd import logfx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    with open(os.path.join(ROOT, "include", "logfx.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(logfx_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(logfx.LIB_PATH):
        pytest.fail("liblogfx.so is not built; run python -m paper_1304_3992_amd.build")
    return logfx.load()


def test_exports_every_declared_symbol(lib):
    names = _declared_functions()
    assert len(names) >= 8
    for n in names:
        assert hasattr(lib, n), f"{n} declared in logfx.h but not exported"
    assert set(logfx.EXPORTS) == set(names)


def test_version(lib):
    assert "liblogfx" in logfx.version()


@pytest.mark.parametrize("size,sigma", [(1, 1.0), (3, 0.5), (5, 0.8), (7, 1.0), (9, 1.4),
                                        (11, 2.0), (15, 3.0)])
@pytest.mark.parametrize("bits", [8, 16, 23])
def test_library_masks_equal_oracle_masks(lib, size, sigma, bits):
    """Each side builds its masks from eq. (1) on its own; they must agree bit
    for bit so that both sides run the same problem."""
    if size == 1:
        with pytest.raises(Exception):
            oracle.log_mask(size, sigma, bits)
        with pytest.raises(logfx.LogfxError):
            logfx.make_log_mask(size, sigma, bits)
        return
    a, ua = oracle.log_mask(size, sigma, bits)
    b, ub = logfx.make_log_mask(size, sigma, bits)
    assert ua == ub
    assert a.tobytes() == b.tobytes()


def _img(h=16, w=16, dtype=logfx.U8, bits=0, pitch=None):
    im = logfx.logfx_image()
    im.data = 0x1000  # never dereferenced by check_params
    im.dtype, im.bits, im.height, im.width = dtype, bits, h, w
    im.pitch = w if pitch is None else pitch
    return im


def _params(s1=5, g1=0.8, s2=9, g2=1.4, bits=16, **kw):
    return logfx.Params(logfx.make_log_mask(s1, g1, bits)[0], logfx.make_log_mask(s2, g2, bits)[0], **kw)


def _rc(img, params):
    return lib_rc(logfx.load(), img, params)


def lib_rc(lib, img, params):
    path = ctypes.c_int32(-1)
    rc = lib.logfx_check_params(ctypes.byref(img) if img is not None else None,
                                ctypes.byref(params.c) if params is not None else None,
                                ctypes.byref(path))
    return rc, path.value


def test_check_params_paths(lib):
    # 16-bit-grid masks: exact in int32 for 8- and 11-bit pixels, FP64 beyond
    assert _rc(_img(), _params()) == (logfx.OK, logfx.PATH_INT32)
    assert _rc(_img(dtype=logfx.U16, bits=11), _params()) == (logfx.OK, logfx.PATH_INT32)
    assert _rc(_img(dtype=logfx.U16), _params()) == (logfx.OK, logfx.PATH_FP64)
    assert _rc(_img(), _params(bits=23)) == (logfx.OK, logfx.PATH_FP64)


def test_check_params_rejections(lib):
    E, U = logfx.EINVAL, logfx.EUNSUPPORTED
    assert _rc(None, _params())[0] == E
    assert _rc(_img(h=0), _params())[0] == E
    assert _rc(_img(w=0), _params())[0] == E
    assert _rc(_img(pitch=3), _params())[0] == E
    assert _rc(_img(dtype=7), _params())[0] == E
    assert _rc(_img(bits=9), _params())[0] == E
    im = _img()
    im.data = 0
    assert _rc(im, _params())[0] == E
    assert _rc(_img(), _params(std_k=-1.0))[0] == E
    assert _rc(_img(), _params(zc_thresh=-1.0))[0] == E
    assert _rc(_img(), _params(zc_thresh=float("nan")))[0] == E
    assert _rc(_img(), _params(median_size=4))[0] == E
    assert _rc(_img(), _params(std_mode=3))[0] == E
    assert _rc(_img(), _params(flags=2))[0] == E
    assert _rc(_img(), _params(median_cascade=(3, 4)))[0] == E
    assert _rc(_img(), _params(median_cascade=(0, 3)))[0] == E
    assert _rc(_img(), _params(median_cascade=(5, 3, 5)))[0] == logfx.OK
    assert _rc(_img(), _params(std5_max=float("nan")))[0] == E
    assert _rc(_img(), _params(std5_max=2.0)) == (logfx.OK, logfx.PATH_INT32)   # the 5x5 first stage
    p = _params()
    p.c.smooth = 5
    assert _rc(_img(), p)[0] == E
    # mask problems
    even = logfx.Params(np.zeros((4, 4), np.float32), logfx.make_log_mask(5, 0.8)[0])
    assert _rc(_img(), even)[0] == E
    big = logfx.Params(logfx.make_log_mask(11, 2.0)[0], logfx.make_log_mask(5, 0.8)[0])
    assert _rc(_img(), big)[0] == U
    asym = logfx.make_log_mask(5, 0.8)[0].copy()
    asym[0, 1] += asym[0, 1]
    assert _rc(_img(), logfx.Params(asym, logfx.make_log_mask(9, 1.4)[0]))[0] == U
    nan = logfx.make_log_mask(5, 0.8)[0].copy()
    nan[2, 2] = np.nan
    assert _rc(_img(), logfx.Params(nan, logfx.make_log_mask(9, 1.4)[0]))[0] == E
    # taps spread over too many binary orders for exact sums with 16-bit pixels
    wide = np.zeros((3, 3), np.float32)
    wide[1, 1] = 1.0
    wide[0, 1] = wide[1, 0] = wide[1, 2] = wide[2, 1] = np.float32(2.0 ** -40)
    rc = _rc(_img(dtype=logfx.U16), logfx.Params(wide, wide))[0]
    assert rc == U
    assert "exact" in logfx.last_error() or "binary orders" in logfx.last_error()


def test_mask_builder_rejections(lib):
    for args in [(4, 1.0, 16), (0, 1.0, 16), (17, 1.0, 16), (5, 0.0, 16), (5, 1.0, 1),
                 (5, 1.0, 24)]:
        with pytest.raises(logfx.LogfxError):
            logfx.make_log_mask(*args)


def test_create_without_device_fails_cleanly(lib):
    """On a machine without a GPU the context call returns an error code
    instead of aborting."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    ptr = ctypes.c_void_p()
    rc = lib.logfx_create(ctypes.byref(ptr), 0)
    assert rc in (logfx.EDEVICE, logfx.EINVAL)
    assert not ptr
    assert lib.logfx_extract(None, None, None, None, None, None) == logfx.EINVAL
    assert lib.logfx_destroy(None) == logfx.OK


def test_gate_constants_and_smooth_modes(lib):
    """The binding's gate constants match the header; GATE is a valid
    smoothing choice for the argument checks."""
    with open(os.path.join(ROOT, "include", "logfx.h")) as f:
        text = f.read()
    for name, val in (("LOGFX_GATE_NPARAM", logfx.GATE_NPARAM), ("LOGFX_GATE_CELLS", logfx.GATE_CELLS),
                      ("LOGFX_GATE_MAX_BATCH", logfx.GATE_MAX_BATCH)):
        assert re.search(rf"#define {name} {val}\b", text), name
    assert re.search(r"LOGFX_SMOOTH_GATE = 2", text)
    assert re.search(r"LOGFX_OPT_STORE_Z = 5", text) and logfx.OPT_STORE_Z == 5
    assert re.search(r"LOGFX_OPT_PACKED_LOG = 6", text) and logfx.OPT_PACKED_LOG == 6
    from oracle import gate as og
    assert og.NPARAM == logfx.GATE_NPARAM
    p = _params()
    p.c.smooth = logfx.SMOOTH_GATE
    assert _rc(_img(), p) == (logfx.OK, logfx.PATH_INT32)


def test_gate_entry_points_reject_null_context(lib):
    """Every gate call returns EINVAL on a NULL context before it touches a
    device."""
    E = logfx.EINVAL
    theta = np.zeros(logfx.GATE_NPARAM, np.float32)
    tp = theta.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    p = _params()
    im = _img()
    assert lib.logfx_gate_features(None, 1, ctypes.byref(im), ctypes.byref(p.c), None, None) == E
    assert lib.logfx_gate(None, 1, ctypes.byref(im), ctypes.byref(p.c), None, None, None) == E
    assert lib.logfx_gate_set_params(None, tp, logfx.GATE_NPARAM) == E
    assert lib.logfx_gate_get_params(None, tp, logfx.GATE_NPARAM) == E
    assert lib.logfx_gate_load(None, b"/nonexistent") == E
    assert lib.logfx_gate_save(None, b"/nonexistent") == E
    assert lib.logfx_gate_save_state(None, b"/nonexistent") == E
    assert lib.logfx_gate_load_state(None, b"/nonexistent") == E
    assert lib.logfx_gate_forward(None, 1, None, None, None, None) == E
    assert lib.logfx_gate_backward(None, 1, None, None, None, None, None, None) == E
    assert lib.logfx_gate_step(None, None, 1e-3, None) == E
    assert "ctx is NULL" in logfx.last_error()


def _wide_range_masks():
    """The benchmark masks with corner taps of 1e-30: exact FP64 sums would
    need integers far beyond 2^52."""
    m1 = logfx.make_log_mask(5, 0.8)[0].copy()
    m2 = logfx.make_log_mask(9, 1.4)[0].copy()
    for m in (m1, m2):
        n = m.shape[0] - 1
        m[0, 0] = m[0, n] = m[n, 0] = m[n, n] = np.float32(1e-30)
    return m1, m2


def test_allow_inexact_flag(lib):
    """Masks whose taps cannot be summed exactly are refused, unless
    LOGFX_ALLOW_INEXACT is set: then they run on the FP64 path."""
    m1, m2 = _wide_range_masks()
    assert _rc(_img(), logfx.Params(m1, m2))[0] == logfx.EUNSUPPORTED
    assert _rc(_img(), logfx.Params(m1, m2, flags=logfx.ALLOW_INEXACT)) == (logfx.OK, logfx.PATH_FP64)
    # exact masks are unaffected by the flag
    assert _rc(_img(), _params(flags=logfx.ALLOW_INEXACT)) == (logfx.OK, logfx.PATH_INT32)


def test_gate_region_checks(lib):
    """The per-region gate: square regions that tile the image exactly, a
    power-of-two count of them each way, GATE smoothing, no cascade."""
    g = logfx.SMOOTH_GATE
    ok = (logfx.OK, logfx.PATH_INT32)
    assert _rc(_img(1024, 512), _params(smooth=g, gate_region=256)) == ok      # 4 x 2 regions
    assert _rc(_img(128, 128), _params(smooth=g, gate_region=128)) == ok       # one region
    assert _rc(_img(16, 16), _params(smooth=g, gate_region=0)) == ok           # off
    bad = [
        (_img(512, 512), dict(smooth=g, gate_region=-1)),                      # negative
        (_img(512, 512), dict(smooth=True, gate_region=256)),                  # not GATE
        (_img(512, 512), dict(smooth=g, gate_region=256, median_cascade=(3,))),
        (_img(512, 512), dict(smooth=g, gate_region=64)),                      # below 128
        (_img(512, 500), dict(smooth=g, gate_region=250)),                     # 512 % 250 != 0
        (_img(768, 512), dict(smooth=g, gate_region=256)),                     # 3 regions down
        (_img(520, 512), dict(smooth=g, gate_region=256)),                     # ragged
        (_img(1 << 17, 1 << 17, pitch=1 << 17), dict(smooth=g, gate_region=128)),  # 2^20 regions
    ]
    rcs = [_rc(im, _params(**kw))[0] for im, kw in bad]
    assert rcs == [logfx.EINVAL] * len(bad), rcs
