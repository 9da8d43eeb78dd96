"""logfx_extract_noalloc, the entry point that allocates nothing (its
scratch is a static device array), called through the C ABI and checked
against logfx_extract on the same inputs: the output bytes must be equal
(both run the same kernels on the same exact sums).  Two calls in a row,
the second on a smaller image, so that the shared array's leftovers from
the first call cannot leak into the second; the limits are refused before
anything is enqueued."""
import ctypes

import pytest

from paper_1304_3992_amd import logfx, scenes
from parity import masks, to_device

pytestmark = pytest.mark.gpu


def _call(lib, ctx, img_t, params, out, bits):
    im = logfx.image(img_t, bits)
    return lib.logfx_extract_noalloc(ctx.ptr, ctypes.byref(im), ctypes.byref(params.c),
                                     ctypes.c_void_p(out.data_ptr()), None)


@pytest.mark.parametrize("smooth", [True, False])
def test_noalloc_equals_extract(smooth):
    import torch
    lib = logfx.load()
    _, lib_t = masks()
    params = logfx.Params(*lib_t, smooth=smooth)
    cases = [(scenes.config2(), 11), (scenes.config1(), 8)]     # 8192^2 11-bit, then 512^2 8-bit
    with logfx.Context(0) as ctx:
        for img, bits in cases:
            d = to_device(img)
            ref = ctx.extract(d, params, bits=bits)
            out = torch.full(img.shape, 0xAB, dtype=torch.uint8, device="cuda")
            torch.cuda.synchronize()
            assert _call(lib, ctx, d, params, out, bits) == logfx.OK, logfx.last_error(ctx.ptr)
            torch.cuda.synchronize()
            assert torch.equal(out, ref), (img.shape, int((out != ref).sum()))
            del d, ref, out
            torch.cuda.empty_cache()


def test_noalloc_fp64_path_and_ragged():
    """The FP64 path (16-bit pixels) and a ragged size that leaves partial
    tiles in both passes."""
    import numpy as np
    import torch
    lib = logfx.load()
    _, lib_t = masks()
    params = logfx.Params(*lib_t)
    img = np.random.default_rng(5).integers(0, 65536, (613, 1037)).astype(np.uint16)
    with logfx.Context(0) as ctx:
        d = to_device(img)
        ref, rep = ctx.extract(d, params, bits=16, report=True)
        assert rep["path"] == logfx.PATH_FP64
        out = torch.full(img.shape, 0xAB, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        assert _call(lib, ctx, d, params, out, 16) == logfx.OK, logfx.last_error(ctx.ptr)
        torch.cuda.synchronize()
        assert torch.equal(out, ref)


def test_noalloc_limits_refused():
    import torch
    lib = logfx.load()
    _, lib_t = masks()
    small = torch.zeros((64, 64), dtype=torch.int16, device="cuda")
    out = torch.zeros((64, 64), dtype=torch.uint8, device="cuda")
    with logfx.Context(0) as ctx:
        # too many tiles: a 33000 x 33000 descriptor (never read: refused first)
        im = logfx.image(small, 11)
        im.height, im.width, im.pitch = 33000, 33000, 33000
        p = logfx.Params(*lib_t)
        rc = lib.logfx_extract_noalloc(ctx.ptr, ctypes.byref(im), ctypes.byref(p.c),
                                       ctypes.c_void_p(out.data_ptr()), None)
        assert rc == logfx.EINVAL and "static scratch" in logfx.last_error(ctx.ptr)
        for kw in (dict(std5_max=1.0), dict(median_cascade=(3,))):
            p = logfx.Params(*lib_t, **kw)
            assert _call(lib, ctx, small, p, out, 11) == logfx.EINVAL
        # the gate with parameters needs context memory; without, GATE runs as ALWAYS
        p = logfx.Params(*lib_t, smooth=logfx.SMOOTH_GATE)
        ref = ctx.extract(small, logfx.Params(*lib_t), bits=11)
        assert _call(lib, ctx, small, p, out, 11) == logfx.OK
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
        from oracle import gate as og
        ctx.gate_set_params(og.init(0))
        assert _call(lib, ctx, small, p, out, 11) == logfx.EINVAL
