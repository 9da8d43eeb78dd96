"""Test infrastructure: the CPU oracle of the LoG feature-extraction pipeline.

Not part of the product.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU library (``paper_1304_3992_amd``); the two are compared by the
tests.

The arithmetic lives in ``logfx_oracle.c`` (plain C, FP64, one function per
stage, each citing the paper passage it follows).  This module only builds it
with gcc and marshals numpy arrays through ctypes.  ``brute`` holds an
independent exact-rational Python version for tiny inputs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "logfx_oracle.c")
_LIB = os.path.join(_HERE, "liblogfx_oracle.so")
_lib = None

U8, U16 = 0, 1
STD_REL, STD_ABS = 0, 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (strict IEEE FP64: no fast-math, no FMA
    contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fno-fast-math", "-ffp-contract=off",
            "-fPIC", "-shared", "-pthread", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        L_, I_, D_ = ctypes.c_long, ctypes.c_int, ctypes.c_double
        lib.orc_log_value.restype = D_
        lib.orc_log_value.argtypes = [D_, D_, D_]
        lib.orc_log_mask.restype = I_
        lib.orc_log_mask.argtypes = [I_, D_, I_, P, P]
        lib.orc_log_response.restype = None
        lib.orc_log_response.argtypes = [P, I_, L_, L_, L_, P, I_, P, I_]
        lib.orc_zero_cross.restype = None
        lib.orc_zero_cross.argtypes = [P, L_, L_, D_, P, I_]
        lib.orc_global_std.restype = D_
        lib.orc_global_std.argtypes = [P, L_]
        lib.orc_local_std.restype = None
        lib.orc_local_std.argtypes = [P, L_, L_, I_, P, I_]
        lib.orc_hybrid_median.restype = None
        lib.orc_hybrid_median.argtypes = [P, L_, L_, I_, P, I_]
        lib.orc_extract.restype = I_
        lib.orc_extract.argtypes = [P, I_, L_, L_, L_, P, I_, P, I_, D_, I_, D_, D_, I_, I_,
                                    P, P, P, P, P, P, P, P, P, I_]
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _dtype_code(img: np.ndarray) -> int:
    if img.dtype == np.uint8:
        return U8
    if img.dtype == np.uint16:
        return U16
    raise TypeError(f"oracle images are uint8 or uint16, got {img.dtype}")


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def log_value(x: float, y: float, sigma: float) -> float:
    """Eq. (1) at one point."""
    return _load().orc_log_value(float(x), float(y), float(sigma))


def log_mask(size: int, sigma: float, grid_bits: int = 16):
    """Zero-sum LoG mask on a power-of-two grid; returns (taps float32 size x size, unit u)."""
    taps = np.zeros((size, size), np.float32)
    u = ctypes.c_double(0.0)
    rc = _load().orc_log_mask(int(size), float(sigma), int(grid_bits), _ptr(taps), ctypes.byref(u))
    if rc != 0:
        raise ValueError(f"invalid mask request size={size} sigma={sigma} grid_bits={grid_bits}")
    return taps, u.value


def log_response(img: np.ndarray, taps: np.ndarray, nthreads: int | None = None) -> np.ndarray:
    img = np.ascontiguousarray(img)
    taps = np.ascontiguousarray(taps, dtype=np.float32)
    H, W = img.shape
    L = np.empty((H, W), np.float64)
    _load().orc_log_response(_ptr(img), _dtype_code(img), H, W, W, _ptr(taps), taps.shape[0],
                             _ptr(L), nthreads or default_threads())
    return L


def zero_cross(L: np.ndarray, zc_thresh: float = 0.0, nthreads: int | None = None) -> np.ndarray:
    L = np.ascontiguousarray(L, dtype=np.float64)
    H, W = L.shape
    Z = np.empty_like(L)
    _load().orc_zero_cross(_ptr(L), H, W, float(zc_thresh), _ptr(Z), nthreads or default_threads())
    return Z


def global_std(Z: np.ndarray) -> float:
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    return _load().orc_global_std(_ptr(Z), Z.size)


def local_std(Z: np.ndarray, win: int = 3, nthreads: int | None = None) -> np.ndarray:
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    H, W = Z.shape
    S = np.empty_like(Z)
    _load().orc_local_std(_ptr(Z), H, W, int(win), _ptr(S), nthreads or default_threads())
    return S


def hybrid_median(E: np.ndarray, win: int = 5, nthreads: int | None = None) -> np.ndarray:
    E = np.ascontiguousarray(E, dtype=np.uint8)
    H, W = E.shape
    F = np.empty_like(E)
    _load().orc_hybrid_median(_ptr(E), H, W, int(win), _ptr(F), nthreads or default_threads())
    return F


def extract(img: np.ndarray, taps1: np.ndarray, taps2: np.ndarray, *, zc_thresh: float = 0.0,
            std_mode: int = STD_REL, std_k: float = 2.0, std5_max: float = -1.0,
            smooth: bool = True, median_size: int = 5, want_intermediates: bool = False,
            nthreads: int | None = None):
    """Run the whole pipeline.  Returns a dict with 'F' (uint8 0/1 map), 'stats'
    (sigma_g1, sigma_g2, T1, T2) and, if requested, 'E', 'L1', 'L2', 'Z1',
    'Z2', 'S1', 'S2'."""
    img = np.ascontiguousarray(img)
    t1 = np.ascontiguousarray(taps1, dtype=np.float32)
    t2 = np.ascontiguousarray(taps2, dtype=np.float32)
    H, W = img.shape
    F = np.empty((H, W), np.uint8)
    stats = np.zeros(4, np.float64)
    inter = {}
    if want_intermediates:
        inter["E"] = np.empty((H, W), np.uint8)
        for k in ("L1", "L2", "Z1", "Z2", "S1", "S2"):
            inter[k] = np.empty((H, W), np.float64)
    g = inter.get
    rc = _load().orc_extract(
        _ptr(img), _dtype_code(img), H, W, W, _ptr(t1), t1.shape[0], _ptr(t2), t2.shape[0],
        float(zc_thresh), int(std_mode), float(std_k), float(std5_max), int(bool(smooth)),
        int(median_size), _ptr(F), _ptr(g("E")), _ptr(g("L1")), _ptr(g("L2")), _ptr(g("Z1")),
        _ptr(g("Z2")), _ptr(g("S1")), _ptr(g("S2")), _ptr(stats), nthreads or default_threads())
    if rc != 0:
        raise RuntimeError(f"oracle extract failed rc={rc}")
    out = {"F": F, "stats": stats}
    out.update(inter)
    return out
