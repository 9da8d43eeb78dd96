"""ctypes binding of liblogfx (include/logfx.h), same names as the C ABI.

Argument marshalling only: every step of the pipeline runs in the HIP
kernels of ``liblogfx.so``.  torch provides device memory and streams.  The
binding fails loudly when the library has not been built; there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblogfx.so")

OK, EINVAL, EUNSUPPORTED, ENOMEM, EDEVICE = 0, 1, 2, 3, 4
U8, U16 = 0, 1
STD_REL, STD_ABS = 0, 1
SMOOTH_NEVER, SMOOTH_ALWAYS, SMOOTH_GATE = 0, 1, 2
PATH_INT32, PATH_FP64 = 0, 1

EXPORTS = ["logfx_version", "logfx_create", "logfx_destroy", "logfx_last_error",
           "logfx_make_log_mask", "logfx_check_params", "logfx_extract", "logfx_extract_maps",
           "logfx_timing_enable", "logfx_timing_read", "logfx_extract_batch",
           "logfx_set_option", "logfx_get_option", "logfx_tune",
           "logfx_gate_features", "logfx_gate_set_params", "logfx_gate_get_params",
           "logfx_gate_load", "logfx_gate_save", "logfx_gate_forward", "logfx_gate_backward",
           "logfx_gate_step", "logfx_gate", "logfx_gate_save_state", "logfx_gate_load_state",
           "logfx_extract_noalloc"]
GATE_NPARAM, GATE_CELLS, GATE_MAX_BATCH = 14369, 128, 4096
OPT_ROWS1, OPT_ROWS2, OPT_PERSISTENT, OPT_GRAPH, OPT_STORE_Z, OPT_PACKED_LOG = 1, 2, 3, 4, 5, 6
ALLOW_INEXACT = 1


class LogfxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"liblogfx error {code}: {msg}")
        self.code = code


class logfx_image(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("dtype", ctypes.c_int32), ("bits", ctypes.c_int32),
                ("height", ctypes.c_int64), ("width", ctypes.c_int64), ("pitch", ctypes.c_int64)]


class logfx_mask(ctypes.Structure):
    _fields_ = [("size", ctypes.c_int32), ("taps", ctypes.POINTER(ctypes.c_float))]


class logfx_params(ctypes.Structure):
    _fields_ = [("mask", logfx_mask * 2), ("zc_thresh", ctypes.c_double),
                ("std_mode", ctypes.c_int32), ("std_k", ctypes.c_double),
                ("std5_max", ctypes.c_double), ("smooth", ctypes.c_int32),
                ("median_size", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("median_cascade", ctypes.c_int32 * 3), ("gate_region", ctypes.c_int32)]


class logfx_tune_result(ctypes.Structure):
    _fields_ = [("rows1", ctypes.c_int32), ("rows2", ctypes.c_int32),
                ("persistent", ctypes.c_int32), ("from_cache", ctypes.c_int32),
                ("ms", ctypes.c_double)]


class logfx_report(ctypes.Structure):
    _fields_ = [("pixels", ctypes.c_int64), ("sigma_g", ctypes.c_double * 2),
                ("thresh", ctypes.c_double * 2), ("zc_count", ctypes.c_int64 * 2),
                ("extracted", ctypes.c_int64), ("output", ctypes.c_int64),
                ("path", ctypes.c_int32), ("smoothed", ctypes.c_int32),
                ("gated", ctypes.c_int32), ("gate_fallback", ctypes.c_int32),
                ("gate_logit", ctypes.c_double), ("inexact", ctypes.c_int32),
                ("regions", ctypes.c_int32), ("regions_smoothed", ctypes.c_int32)]

    def as_dict(self):
        return {"pixels": self.pixels, "sigma_g": list(self.sigma_g), "thresh": list(self.thresh),
                "zc_count": list(self.zc_count), "extracted": self.extracted,
                "output": self.output, "path": self.path, "smoothed": self.smoothed,
                "gated": self.gated, "gate_fallback": self.gate_fallback,
                "gate_logit": self.gate_logit, "inexact": self.inexact,
                "regions": self.regions, "regions_smoothed": self.regions_smoothed}


_lib = None


def load(path: str | None = None):
    """Load liblogfx.so (torch is imported first so that one HIP runtime
    serves both)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"liblogfx.so not built ({path}); run `python -m paper_1304_3992_amd.build`")
    try:
        import torch  # noqa: F401  (loads the HIP runtime torch was built with)
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.logfx_version.restype = ctypes.c_char_p
    lib.logfx_version.argtypes = []
    lib.logfx_create.restype = ctypes.c_int
    lib.logfx_create.argtypes = [ctypes.POINTER(P), ctypes.c_int]
    lib.logfx_destroy.restype = ctypes.c_int
    lib.logfx_destroy.argtypes = [P]
    lib.logfx_last_error.restype = ctypes.c_char_p
    lib.logfx_last_error.argtypes = [P]
    lib.logfx_make_log_mask.restype = ctypes.c_int
    lib.logfx_make_log_mask.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_float),
                                        ctypes.POINTER(ctypes.c_double)]
    lib.logfx_check_params.restype = ctypes.c_int
    lib.logfx_check_params.argtypes = [ctypes.POINTER(logfx_image), ctypes.POINTER(logfx_params),
                                       ctypes.POINTER(ctypes.c_int32)]
    lib.logfx_extract.restype = ctypes.c_int
    lib.logfx_extract.argtypes = [P, ctypes.POINTER(logfx_image), ctypes.POINTER(logfx_params), P,
                                  ctypes.POINTER(logfx_report), P]
    lib.logfx_extract_noalloc.restype = ctypes.c_int
    lib.logfx_extract_noalloc.argtypes = [P, ctypes.POINTER(logfx_image), ctypes.POINTER(logfx_params), P, P]
    lib.logfx_extract_maps.restype = ctypes.c_int
    lib.logfx_extract_maps.argtypes = [P, ctypes.POINTER(logfx_image),
                                       ctypes.POINTER(logfx_params), P, P, P, P, P]
    lib.logfx_extract_batch.restype = ctypes.c_int
    lib.logfx_extract_batch.argtypes = [P, ctypes.c_int32, ctypes.POINTER(logfx_image),
                                        ctypes.POINTER(logfx_params), ctypes.POINTER(P),
                                        ctypes.POINTER(logfx_report), P]
    lib.logfx_set_option.restype = ctypes.c_int
    lib.logfx_set_option.argtypes = [P, ctypes.c_int32, ctypes.c_int64]
    lib.logfx_get_option.restype = ctypes.c_int
    lib.logfx_get_option.argtypes = [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]
    lib.logfx_tune.restype = ctypes.c_int
    lib.logfx_tune.argtypes = [P, ctypes.c_int32, ctypes.POINTER(logfx_image),
                               ctypes.POINTER(logfx_params), ctypes.POINTER(P), ctypes.c_int32,
                               ctypes.c_char_p, ctypes.POINTER(logfx_tune_result), P]
    lib.logfx_timing_enable.restype = ctypes.c_int
    lib.logfx_timing_enable.argtypes = [P, ctypes.c_int]
    lib.logfx_timing_read.restype = ctypes.c_int
    lib.logfx_timing_read.argtypes = [P, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_int64)]
    IMGS, PAR = ctypes.POINTER(logfx_image), ctypes.POINTER(logfx_params)
    FP = ctypes.POINTER(ctypes.c_float)
    for name, args in [
            ("logfx_gate_features", [P, ctypes.c_int32, IMGS, PAR, P, P]),
            ("logfx_gate_set_params", [P, FP, ctypes.c_int64]),
            ("logfx_gate_get_params", [P, FP, ctypes.c_int64]),
            ("logfx_gate_load", [P, ctypes.c_char_p]),
            ("logfx_gate_save", [P, ctypes.c_char_p]),
            ("logfx_gate_save_state", [P, ctypes.c_char_p]),
            ("logfx_gate_load_state", [P, ctypes.c_char_p]),
            ("logfx_gate_forward", [P, ctypes.c_int32, P, P, P, P]),
            ("logfx_gate_backward", [P, ctypes.c_int32, P, P, P, P, P, P]),
            ("logfx_gate_step", [P, P, ctypes.c_double, P]),
            ("logfx_gate", [P, ctypes.c_int32, IMGS, PAR, P, P, P])]:
        getattr(lib, name).restype = ctypes.c_int
        getattr(lib, name).argtypes = args
    _lib = lib
    return lib


def version() -> str:
    return load().logfx_version().decode()


def last_error(ctx=None) -> str:
    msg = load().logfx_last_error(ctx)
    return msg.decode() if msg else ""


def _check(rc, ctx=None):
    if rc != OK:
        raise LogfxError(rc, last_error(ctx))


def make_log_mask(size: int, sigma: float, grid_bits: int = 16):
    """logfx_make_log_mask: returns (taps float32 [size, size], unit)."""
    taps = np.zeros((size, size), np.float32)
    unit = ctypes.c_double(0.0)
    lib = load()
    _check(lib.logfx_make_log_mask(size, sigma, grid_bits,
                                   taps.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                   ctypes.byref(unit)))
    return taps, unit.value


class Params:
    """Holds a logfx_params struct and keeps its tap arrays alive."""

    def __init__(self, taps1, taps2, *, zc_thresh=0.0, std_mode=STD_REL, std_k=2.0,
                 std5_max=-1.0, smooth=True, median_size=5, flags=0, median_cascade=(), gate_region=0):
        self.t1 = np.ascontiguousarray(taps1, dtype=np.float32)
        self.t2 = np.ascontiguousarray(taps2, dtype=np.float32)
        p = logfx_params()
        for i, t in enumerate((self.t1, self.t2)):
            p.mask[i].size = t.shape[0]
            p.mask[i].taps = t.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        p.zc_thresh = zc_thresh
        p.std_mode = std_mode
        p.std_k = std_k
        p.std5_max = std5_max
        # True / False, or one of SMOOTH_NEVER / SMOOTH_ALWAYS / SMOOTH_GATE
        p.smooth = smooth if not isinstance(smooth, bool) else (SMOOTH_ALWAYS if smooth else SMOOTH_NEVER)
        p.median_size = median_size
        p.flags = flags
        cas = list(median_cascade)
        if len(cas) > 3:
            raise ValueError("at most 3 further median levels")
        for i, m in enumerate(cas + [0] * (3 - len(cas))):
            p.median_cascade[i] = m
        p.gate_region = gate_region
        self.c = p


def _feature_sets(imgs, params: Params) -> int:
    """Images, or regions of the single image when params.gate_region > 0."""
    r = params.c.gate_region
    if r > 0 and len(imgs) == 1 and imgs[0].shape[0] % r == 0 and imgs[0].shape[1] % r == 0:
        return (imgs[0].shape[0] // r) * (imgs[0].shape[1] // r)
    return len(imgs)   # the library rejects any other region geometry


def _torch_dtype_code(t) -> int:
    import torch
    if t.dtype == torch.uint8:
        return U8
    if t.dtype in (torch.int16, torch.uint16):
        return U16
    raise TypeError(f"images are uint8 or 16-bit tensors, got {t.dtype}")


def image(t, bits: int = 0) -> logfx_image:
    """Describe a 2-D device tensor (uint8, or int16/uint16 holding 16-bit
    pixels); the row stride of the tensor is the pitch."""
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError("image must be a 2-D tensor with unit column stride")
    im = logfx_image()
    im.data = t.data_ptr()
    im.dtype = _torch_dtype_code(t)
    im.bits = bits
    im.height, im.width = t.shape
    im.pitch = t.stride(0)
    return im


def check_params(img: logfx_image, params: Params) -> int:
    path = ctypes.c_int32(-1)
    _check(load().logfx_check_params(ctypes.byref(img), ctypes.byref(params.c), ctypes.byref(path)))
    return path.value


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Context:
    """Owns a logfx_ctx on one device."""

    def __init__(self, device: int = 0):
        self.lib = load()
        self.ptr = ctypes.c_void_p()
        _check(self.lib.logfx_create(ctypes.byref(self.ptr), device))
        self.device = device

    def close(self):
        if self.ptr:
            self.lib.logfx_destroy(self.ptr)
            self.ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def extract(self, img_t, params: Params, out=None, *, bits: int = 0, report: bool = False,
                stream=None):
        """logfx_extract on a device tensor; returns the uint8 map (and the
        report dict when ``report``)."""
        import torch
        img = image(img_t, bits)
        if out is None:
            out = torch.empty(img_t.shape, dtype=torch.uint8, device=img_t.device)
        rep = logfx_report() if report else None
        rc = self.lib.logfx_extract(self.ptr, ctypes.byref(img), ctypes.byref(params.c),
                                    ctypes.c_void_p(out.data_ptr()),
                                    ctypes.byref(rep) if rep is not None else None,
                                    _stream_ptr(stream))
        _check(rc, self.ptr)
        return (out, rep.as_dict()) if report else out

    def extract_noalloc(self, img_t, params: Params, out, *, bits: int = 0, stream=None):
        """logfx_extract_noalloc: the pipeline into the caller's uint8 map
        `out` (same shape as the image) with no allocation in the library."""
        img = image(img_t, bits)
        rc = self.lib.logfx_extract_noalloc(self.ptr, ctypes.byref(img), ctypes.byref(params.c),
                                            ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream))
        _check(rc, self.ptr)
        return out

    def timing_enable(self, on: bool = True):
        _check(self.lib.logfx_timing_enable(self.ptr, int(bool(on))), self.ptr)

    def timing_read(self):
        """Summed milliseconds (pass 1, finalize, pass 2, whole call) and the
        number of timed calls since the last read."""
        ms = (ctypes.c_double * 4)()
        calls = ctypes.c_int64(0)
        _check(self.lib.logfx_timing_read(self.ptr, ms, ctypes.byref(calls)), self.ptr)
        return list(ms), calls.value

    def set_option(self, option: int, value: int):
        _check(self.lib.logfx_set_option(self.ptr, option, int(value)), self.ptr)

    def get_option(self, option: int) -> int:
        v = ctypes.c_int64(0)
        _check(self.lib.logfx_get_option(self.ptr, option, ctypes.byref(v)), self.ptr)
        return v.value

    def extract_batch(self, imgs, params: Params, outs=None, *, bits: int = 0,
                      report: bool = False, stream=None):
        """logfx_extract_batch on a list of device tensors; returns the list of
        uint8 maps (and the list of report dicts when ``report``)."""
        import torch
        n = len(imgs)
        descs = (logfx_image * n)(*[image(t, bits) for t in imgs])
        if outs is None:
            outs = [torch.empty(t.shape, dtype=torch.uint8, device=t.device) for t in imgs]
        ptrs = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
        reps = (logfx_report * n)() if report else None
        rc = self.lib.logfx_extract_batch(self.ptr, n, descs, ctypes.byref(params.c), ptrs,
                                          reps, _stream_ptr(stream))
        _check(rc, self.ptr)
        return (outs, [r.as_dict() for r in reps]) if report else outs

    def tune(self, imgs, params: Params, outs=None, *, bits: int = 0, reps: int = 5,
             cache: str | None = None, stream=None) -> dict:
        """logfx_tune for one image (a tensor) or a batch (a list of tensors)."""
        import torch
        imgs = list(imgs) if isinstance(imgs, (list, tuple)) else [imgs]
        n = len(imgs)
        descs = (logfx_image * n)(*[image(t, bits) for t in imgs])
        if outs is None:
            outs = [torch.empty(t.shape, dtype=torch.uint8, device=t.device) for t in imgs]
        ptrs = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
        res = logfx_tune_result()
        rc = self.lib.logfx_tune(self.ptr, n, descs, ctypes.byref(params.c), ptrs, reps,
                                 cache.encode() if cache else None, ctypes.byref(res),
                                 _stream_ptr(stream))
        _check(rc, self.ptr)
        return {"rows1": res.rows1, "rows2": res.rows2, "persistent": res.persistent,
                "from_cache": res.from_cache, "ms": res.ms}

    def extract_maps(self, img_t, params: Params, *, bits: int = 0, want=("L1", "L2", "Z1", "Z2"),
                     stream=None):
        """logfx_extract_maps: returns a dict of FP64 device maps."""
        import torch
        img = image(img_t, bits)
        outs = {k: torch.empty(img_t.shape, dtype=torch.float64, device=img_t.device)
                for k in want}
        ptr = [ctypes.c_void_p(outs[k].data_ptr()) if k in outs else None
               for k in ("L1", "L2", "Z1", "Z2")]
        rc = self.lib.logfx_extract_maps(self.ptr, ctypes.byref(img), ctypes.byref(params.c),
                                         *ptr, _stream_ptr(stream))
        _check(rc, self.ptr)
        return outs

    # ------------------------------------------------------------ gate
    def _descs(self, imgs, bits):
        imgs = list(imgs) if isinstance(imgs, (list, tuple)) else [imgs]
        return imgs, (logfx_image * len(imgs))(*[image(t, bits) for t in imgs])

    def gate_features(self, imgs, params: Params, feats=None, *, bits: int = 0, stream=None):
        """logfx_gate_features: bfloat16 features [n, 3, 128, 128] on the device."""
        import torch
        imgs, descs = self._descs(imgs, bits)
        n = len(imgs)
        if feats is None:
            sets = _feature_sets(imgs, params)
            feats = torch.empty((sets, 3, GATE_CELLS, GATE_CELLS), dtype=torch.bfloat16, device=imgs[0].device)
        rc = self.lib.logfx_gate_features(self.ptr, n, descs, ctypes.byref(params.c),
                                          ctypes.c_void_p(feats.data_ptr()), _stream_ptr(stream))
        _check(rc, self.ptr)
        return feats

    def gate_set_params(self, theta):
        t = np.ascontiguousarray(theta, dtype=np.float32)
        _check(self.lib.logfx_gate_set_params(self.ptr, t.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                              t.size), self.ptr)

    def gate_get_params(self):
        t = np.zeros(GATE_NPARAM, np.float32)
        _check(self.lib.logfx_gate_get_params(self.ptr, t.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                              t.size), self.ptr)
        return t

    def gate_load(self, path: str):
        _check(self.lib.logfx_gate_load(self.ptr, os.fsencode(path)), self.ptr)

    def gate_save(self, path: str):
        _check(self.lib.logfx_gate_save(self.ptr, os.fsencode(path)), self.ptr)

    def gate_save_state(self, path: str):
        _check(self.lib.logfx_gate_save_state(self.ptr, os.fsencode(path)), self.ptr)

    def gate_load_state(self, path: str):
        _check(self.lib.logfx_gate_load_state(self.ptr, os.fsencode(path)), self.ptr)

    @staticmethod
    def _batch(feats, idx, B):
        if idx is not None:
            return int(idx.numel()), ctypes.c_void_p(idx.data_ptr())
        return int(B if B is not None else feats.shape[0]), None

    def gate_forward(self, feats, idx=None, *, B=None, logits=None, stream=None):
        """Logits of the samples (all of feats, the first B, or feats[idx])."""
        import torch
        nb, ip = self._batch(feats, idx, B)
        if logits is None:
            logits = torch.empty(nb, dtype=torch.float32, device=feats.device)
        rc = self.lib.logfx_gate_forward(self.ptr, nb, ctypes.c_void_p(feats.data_ptr()), ip,
                                         ctypes.c_void_p(logits.data_ptr()), _stream_ptr(stream))
        _check(rc, self.ptr)
        return logits

    def gate_backward(self, feats, labels, idx=None, *, B=None, grad=None, loss=None, stream=None):
        """(gradient [GATE_NPARAM], mean loss [1]) as device float tensors.
        grad=False leaves the gradient in the context's buffer for gate_step."""
        import torch
        nb, ip = self._batch(feats, idx, B)
        if grad is None:
            grad = torch.empty(GATE_NPARAM, dtype=torch.float32, device=feats.device)
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device=feats.device)
        gp = None if grad is False else ctypes.c_void_p(grad.data_ptr())
        rc = self.lib.logfx_gate_backward(self.ptr, nb, ctypes.c_void_p(feats.data_ptr()), ip,
                                          ctypes.c_void_p(labels.data_ptr()), gp,
                                          ctypes.c_void_p(loss.data_ptr()), _stream_ptr(stream))
        _check(rc, self.ptr)
        return (None if grad is False else grad), loss

    def gate_step(self, lr: float, grad=None, *, stream=None):
        gp = None if grad is None else ctypes.c_void_p(grad.data_ptr())
        _check(self.lib.logfx_gate_step(self.ptr, gp, float(lr), _stream_ptr(stream)), self.ptr)

    def gate(self, imgs, params: Params, *, bits: int = 0, stream=None):
        """logfx_gate: (logits float [n], decisions uint8 [n]) device tensors
        (one per region, row-major, when params.gate_region > 0)."""
        import torch
        imgs, descs = self._descs(imgs, bits)
        n = len(imgs)
        sets = _feature_sets(imgs, params)
        logits = torch.empty(sets, dtype=torch.float32, device=imgs[0].device)
        dec = torch.empty(sets, dtype=torch.uint8, device=imgs[0].device)
        rc = self.lib.logfx_gate(self.ptr, n, descs, ctypes.byref(params.c),
                                 ctypes.c_void_p(logits.data_ptr()), ctypes.c_void_p(dec.data_ptr()),
                                 _stream_ptr(stream))
        _check(rc, self.ptr)
        return logits, dec
