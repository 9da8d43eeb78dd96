"""Seeded synthetic scenes standing in for the paper's satellite images.

The paper's inputs (Cartosat-1 panchromatic scenes of 2000^2 and 4000^2
pixels, and 12-bit Resourcesat-2 AWiFS bands, Sec. 6) are not available, so
every workload is generated here from a seed.  This module holds no
arithmetic of the feature-extraction method: it only draws pixels.  Both the
GPU tests and the oracle tests take their images from it.

Recipe (one panchromatic band):
  * background 60 + 80 t, with t in [0, 1] the normalised projection of the
    pixel position on a random direction;
  * axis-aligned rectangles, sides uniform integers in [8, 64], top-left corner
    uniform in the image (clipped at the border), value uniform integer in
    [150, 250]; later rectangles overwrite earlier ones;
  * polylines of 2-6 random vertices and width 1, 2 or 3 px: a pixel is on
    the line when its distance to a segment is at most width/2; value as for
    rectangles;
  * values are scaled by (2^bits - 1)/255 for deeper images, Gaussian noise
    N(0, sigma^2) is added, rounded half to even and clipped to
    [0, 2^bits - 1];
  * salt-and-pepper impulses with density p, half at 0 and half at the
    maximum value.
"""
from __future__ import annotations

import hashlib
import math

import numpy as np


def _polyline(img: np.ndarray, rng: np.random.Generator, value: float) -> None:
    H, W = img.shape
    nv = int(rng.integers(2, 7))
    width = int(rng.integers(1, 4))
    pts = np.stack([rng.uniform(0, H - 1, nv), rng.uniform(0, W - 1, nv)], axis=1)
    r = width / 2.0
    for (y0, x0), (y1, x1) in zip(pts[:-1], pts[1:]):
        dy, dx = y1 - y0, x1 - x0
        seg2 = dy * dy + dx * dx
        steep = abs(dy) > abs(dx)
        # walk the major axis; test a few candidates across it
        if steep:
            a0, a1, b0, db = y0, y1, x0, dx
        else:
            a0, a1, b0, db = x0, x1, y0, dy
        da = (a1 - a0) if (a1 - a0) != 0 else 1e-12
        lo = int(math.floor(min(a0, a1) - r)) - 1
        hi = int(math.ceil(max(a0, a1) + r)) + 1
        amax = (H if steep else W) - 1
        bmax = (W if steep else H) - 1
        a = np.arange(max(lo, 0), min(hi, amax) + 1)
        if a.size == 0:
            continue
        tpar = np.clip((a - a0) / da, 0.0, 1.0)
        bc = b0 + tpar * db
        span = int(math.ceil(r * math.sqrt(1.0 + (db / da) ** 2))) + 2
        off = np.arange(-span, span + 1)
        A = np.repeat(a, off.size)
        B = (np.round(bc).astype(np.int64)[:, None] + off[None, :]).ravel()
        keep = (B >= 0) & (B <= bmax)
        A, B = A[keep], B[keep]
        Y, X = (A, B) if steep else (B, A)
        if seg2 == 0:
            d2 = (Y - y0) ** 2 + (X - x0) ** 2
        else:
            t = np.clip(((Y - y0) * dy + (X - x0) * dx) / seg2, 0.0, 1.0)
            d2 = (Y - (y0 + t * dy)) ** 2 + (X - (x0 + t * dx)) ** 2
        on = d2 <= r * r + 1e-9
        img[Y[on], X[on]] = value


def panchromatic(height: int, width: int, seed: int, *, n_rect: int = 40, n_poly: int = 0,
                 noise_sigma: float = 4.0, sp_density: float = 0.0, bits: int = 8,
                 dtype=None) -> np.ndarray:
    """One synthetic band.  ``bits`` = 8 gives uint8 unless ``dtype`` says
    otherwise; deeper images are uint16."""
    rng = np.random.default_rng(seed)
    H, W = int(height), int(width)
    maxv = (1 << bits) - 1
    theta = rng.uniform(0.0, 2.0 * math.pi)
    img = np.arange(H, dtype=np.float64)[:, None] * math.sin(theta) + \
        np.arange(W, dtype=np.float64)[None, :] * math.cos(theta)
    lo, hi = img.min(), img.max()
    if hi > lo:
        img -= lo
        img *= 80.0 / (hi - lo)
    else:
        img[:] = 0.0
    img += 60.0
    for _ in range(int(n_rect)):
        h = int(rng.integers(8, 65))
        w = int(rng.integers(8, 65))
        y0 = int(rng.integers(0, H))
        x0 = int(rng.integers(0, W))
        img[y0:y0 + h, x0:x0 + w] = float(rng.integers(150, 251))
    for _ in range(int(n_poly)):
        _polyline(img, rng, float(rng.integers(150, 251)))
    if bits != 8:
        img *= maxv / 255.0
    if noise_sigma > 0:
        img += rng.normal(0.0, noise_sigma, size=img.shape)
    np.rint(img, out=img)
    np.clip(img, 0, maxv, out=img)
    if sp_density > 0:
        u = rng.random(img.shape)
        img[u < sp_density / 2] = 0
        img[(u >= sp_density / 2) & (u < sp_density)] = maxv
    if dtype is None:
        dtype = np.uint8 if bits <= 8 else np.uint16
    return img.astype(dtype)


def config1(seed: int = 1) -> np.ndarray:
    """512 x 512 uint8, 40 rectangles, noise sigma 4."""
    return panchromatic(512, 512, seed, n_rect=40, noise_sigma=4.0, bits=8)


def config2(seed: int = 2, size: int = 8192) -> np.ndarray:
    """8192 x 8192 uint16 11-bit: 20000 rectangles, 500 polylines, sigma 12,
    5 % salt-and-pepper at 0/2047.  ``size`` scales the scene (rectangle and
    polyline counts scale with the area) for smaller test cases."""
    scale = (size * size) / float(8192 * 8192)
    return panchromatic(size, size, seed, n_rect=max(1, round(20000 * scale)),
                        n_poly=max(1, round(500 * scale)), noise_sigma=12.0, sp_density=0.05,
                        bits=11)


def tile_shapes(n: int = 64, seed: int = 3, lo: int = 256, hi: int = 4096):
    """Tile sides drawn log-uniform in [lo, hi], height and width independent."""
    rng = np.random.default_rng(seed)
    ll, lh = math.log(lo), math.log(hi)
    hs = np.clip(np.round(np.exp(rng.uniform(ll, lh, n))), lo, hi).astype(int)
    ws = np.clip(np.round(np.exp(rng.uniform(ll, lh, n))), lo, hi).astype(int)
    return list(zip(hs.tolist(), ws.tolist()))


def config3(n: int = 64, seed: int = 3, base_seed: int = 3000, lo: int = 256, hi: int = 4096):
    """Uneven tiles, each from the 512^2 generator with its own seed and a
    rectangle count scaled by area (40 per 512^2); uint8 values held in
    uint16."""
    tiles = []
    for i, (h, w) in enumerate(tile_shapes(n, seed, lo, hi)):
        nr = max(1, round(40 * h * w / (512.0 * 512.0)))
        tiles.append(panchromatic(h, w, base_seed + i, n_rect=nr, noise_sigma=4.0, bits=8,
                                  dtype=np.uint16))
    return tiles


def gate_tile(index: int, size: int = 512, base_seed: int = 400000, twin: bool = True,
              band: bool = False):
    """One training tile of the smoothing gate and its noise-free twin: the
    8192^2 generator's density of rectangles and polylines on a size^2 11-bit
    tile, Gaussian noise sigma ~ U[0, 20] and salt-and-pepper density
    ~ U[0, 0.2].  With band, the noise-free tile is first mapped to another
    band as the four-band workload does (round(g * tile + o), clipped, with
    gain g ~ U[0.6, 1.2] and offset o ~ U[-60, 100]) and the noise is added
    to that.  Returns (noisy, clean, sigma, density); clean is None when twin
    is False (and band is False)."""
    rng = np.random.default_rng(base_seed + index)
    sigma = float(rng.uniform(0.0, 20.0))
    density = float(rng.uniform(0.0, 0.2))
    scale = size * size / float(8192 * 8192)
    kw = dict(n_rect=max(1, round(20000 * scale)), n_poly=max(1, round(500 * scale)), bits=11)
    seed = base_seed + 1_000_000 + index
    if band:
        gain, offset = float(rng.uniform(0.6, 1.2)), float(rng.uniform(-60.0, 100.0))
        base = panchromatic(size, size, seed, noise_sigma=0.0, sp_density=0.0, **kw).astype(np.float64)
        clean = np.clip(np.rint(gain * base + offset), 0, 2047)
        noisy = _noise(clean, rng, sigma, density, 2047)
        return noisy, clean.astype(np.uint16), sigma, density
    noisy = panchromatic(size, size, seed, noise_sigma=sigma, sp_density=density, **kw)
    clean = panchromatic(size, size, seed, noise_sigma=0.0, sp_density=0.0, **kw) if twin else None
    return noisy, clean, sigma, density


def _noise(clean: np.ndarray, rng: np.random.Generator, sigma: float, density: float, maxv: int) -> np.ndarray:
    """Gaussian noise (rounded, clipped) then salt-and-pepper impulses on a
    noise-free float image; returns uint16."""
    img = clean + rng.normal(0.0, sigma, size=clean.shape) if sigma > 0 else clean.copy()
    np.rint(img, out=img)
    np.clip(img, 0, maxv, out=img)
    u = rng.random(img.shape)
    img[u < density / 2] = 0
    img[(u >= density / 2) & (u < density)] = maxv
    return img.astype(np.uint16)


def sha256(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


# Four-band workload of the gated pipeline: 16384^2 bands cut into 2048^2
# tiles.  One noise-free base scene (the 8192^2 generator at four times the
# area); band b is round(gain_b * base + offset_b), clipped to 11 bits; each
# (band, tile) gets its own Gaussian noise sigma ~ U[0, 20] and salt-and-
# pepper density ~ U[0, 0.2], so that smoothing helps some tiles and not
# others.
C5_GAIN = (0.9, 1.0, 1.1, 0.7)
C5_OFFSET = (0.0, 40.0, -40.0, 80.0)


def config5_base(size: int = 16384, seed: int = 5) -> np.ndarray:
    scale = size * size / float(8192 * 8192)
    return panchromatic(size, size, seed, n_rect=round(20000 * scale), n_poly=round(500 * scale),
                        noise_sigma=0.0, sp_density=0.0, bits=11)


def config5_tile(base: np.ndarray, band: int, ty: int, tx: int, tile: int = 2048, seed: int = 5,
                 per_band: bool = False):
    """(noisy, clean, sigma, density) of tile (ty, tx) of band `band`.  By
    default every (band, tile) draws its own sigma ~ U[0, 20] and density
    ~ U[0, 0.2]; with per_band the band draws them once for all its tiles
    (the noise of a band as a sensor gives it), and each tile still draws
    its own noise values."""
    maxv = 2047
    rng = np.random.default_rng([seed, band, ty, tx])
    sigma = float(rng.uniform(0.0, 20.0))
    density = float(rng.uniform(0.0, 0.2))
    if per_band:
        brng = np.random.default_rng([seed, 1000 + band])
        sigma = float(brng.uniform(0.0, 20.0))
        density = float(brng.uniform(0.0, 0.2))
    b = base[ty * tile:(ty + 1) * tile, tx * tile:(tx + 1) * tile].astype(np.float64)
    clean = np.clip(np.rint(C5_GAIN[band] * b + C5_OFFSET[band]), 0, maxv)
    return _noise(clean, rng, sigma, density, maxv), clean.astype(np.uint16), sigma, density


def config5_index(size: int = 16384, tile: int = 2048, bands: int = 4):
    """(band, ty, tx) of every tile, in order."""
    n = size // tile
    return [(b, ty, tx) for b in range(bands) for ty in range(n) for tx in range(n)]


def regional_noise_scene(height: int = 4096, width: int = 16384, region: int = 2048, seed: int = 6,
                         bits: int = 11) -> np.ndarray:
    """A noise-free 11-bit scene at the 8192^2 generator's density of
    rectangles and polylines, then each region x region square with its own
    Gaussian noise sigma ~ U[0, 20] and salt-and-pepper density ~ U[0, 0.2]
    (the four-band workload's noise law, on one seamless image)."""
    area = height * width / (8192.0 * 8192.0)
    base = panchromatic(height, width, seed, n_rect=int(20000 * area), n_poly=int(500 * area),
                        noise_sigma=0.0, sp_density=0.0, bits=bits).astype(np.float64)
    rng = np.random.default_rng(seed + 1)
    maxv = (1 << bits) - 1
    out = np.empty((height, width), np.uint16)
    for y in range(0, height, region):
        for x in range(0, width, region):
            sigma, density = float(rng.uniform(0.0, 20.0)), float(rng.uniform(0.0, 0.2))
            out[y:y + region, x:x + region] = _noise(base[y:y + region, x:x + region], rng, sigma, density, maxv)
    return out
