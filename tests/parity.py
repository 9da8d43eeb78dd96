"""Shared helpers of the GPU parity tests: move seeded images to the device,
run the library and the oracle on them, and compare the maps with the band
rule.  No arithmetic of the method lives here."""
from __future__ import annotations

import numpy as np

import oracle
from paper_1304_3992_amd import logfx

# A pixel is a band pixel when the oracle's 3x3 deviation lies within this
# relative distance of its threshold; only there may the GPU decide
# differently (FP64 rounding order).  LoG responses and crossing strengths
# are exact on both sides and must agree bit for bit.
BAND_REL = 1e-5
MISMATCH_BUDGET = 1e-6


def to_device(img: np.ndarray, pitch: int | None = None):
    import torch
    a = np.ascontiguousarray(img)
    if a.dtype == np.uint16:
        a = a.view(np.int16)
    t = torch.from_numpy(a)
    if pitch is not None and pitch > img.shape[1]:
        big = torch.zeros((img.shape[0], pitch), dtype=t.dtype)
        big[:, :img.shape[1]] = t
        return big.cuda()[:, :img.shape[1]]
    return t.cuda()


def masks(pair=((5, 0.8), (9, 1.4)), grid_bits=16):
    """(oracle taps, library taps) for both masks -- each side builds its own."""
    (s1, g1), (s2, g2) = pair
    orc = (oracle.log_mask(s1, g1, grid_bits)[0], oracle.log_mask(s2, g2, grid_bits)[0])
    lib = (logfx.make_log_mask(s1, g1, grid_bits)[0], logfx.make_log_mask(s2, g2, grid_bits)[0])
    return orc, lib


def run_gpu(ctx, img, lib_taps, *, bits=0, pitch=None, report=True, **kw):
    import torch
    t = to_device(img, pitch)
    params = logfx.Params(lib_taps[0], lib_taps[1], **kw)
    res = ctx.extract(t, params, bits=bits, report=report)
    torch.cuda.synchronize()
    if report:
        out, rep = res
        return out.cpu().numpy(), rep
    return res.cpu().numpy(), None


def run_oracle(img, orc_taps, **kw):
    return oracle.extract(img, orc_taps[0], orc_taps[1], want_intermediates=True, **kw)


def band(orc, std5_max: float = -1.0) -> np.ndarray:
    """Band pixels: the oracle's 3x3 deviation (and, with the 5x5 first
    stage, its 5x5 deviation, from the oracle's own local_std of its Z
    maps) within BAND_REL of the threshold."""
    b = np.zeros(orc["F"].shape, bool)
    for j, S in ((0, orc["S1"]), (1, orc["S2"])):
        T = orc["stats"][2 + j]
        if T > 0:
            b |= np.abs(S - T) <= BAND_REL * T
        if std5_max >= 0:
            S5 = oracle.local_std(orc["Z1" if j == 0 else "Z2"], 5)
            b |= np.abs(S5 - std5_max) <= BAND_REL * max(std5_max, 1e-300)
    return b


def dilate(mask: np.ndarray, r: int) -> np.ndarray:
    if r == 0:
        return mask.copy()
    H, W = mask.shape
    P = np.pad(mask, r)
    out = np.zeros_like(mask)
    for dy in range(2 * r + 1):
        for dx in range(2 * r + 1):
            out |= P[dy:dy + H, dx:dx + W]
    return out


def compare(F_gpu: np.ndarray, orc, *, smooth: bool, median_size: int = 5, std5_max: float = -1.0,
            radius: int | None = None) -> dict:
    """Checks the band rule and returns counts.  radius: how far a band
    pixel's decision reaches into the output (default: the median's)."""
    b = band(orc, std5_max)
    ref = orc["F"]
    mism = F_gpu != ref
    excused = dilate(b, radius if radius is not None else (median_size // 2 if smooth else 0))
    unexcused = int((mism & ~excused).sum())
    n = ref.size
    info = {"mismatch": int(mism.sum()), "unexcused": unexcused, "band": int(b.sum()), "n": n}
    assert unexcused == 0, info
    assert info["mismatch"] <= MISMATCH_BUDGET * n, info
    return info
