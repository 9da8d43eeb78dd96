"""Test infrastructure: FP64 oracle of the smoothing gate (features, network,
loss, gradients, AdamW).  Not part of the product; only tests import it.

The paper leaves the choice to smooth or not to the user, who makes it
from how noisy the extracted map is (abstract; Sec. 4).  The gate makes
that choice per tile with a small CNN:

  features  3 x 128 x 128 per tile: per cell (an area-downsample of the tile),
            the mean pixel value / (2^bits - 1) and the fraction of pixels
            whose crossing strength Z_1, Z_2 is non-zero (Sec. 3.2);
  network   conv3x3 stride 2 pad 1 (3->16) ReLU, conv (16->32) ReLU,
            conv (32->32) ReLU  [128 -> 64 -> 32 -> 16], global average
            pool, linear 32 -> 1 logit;
  loss      binary cross-entropy with logits, mean over the batch;
  optimiser AdamW on FP32 master weights;
  labels    smoothing_label / tile_label below: the rule that writes every
            stored training and evaluation label.

The GPU keeps the features, the convolution weights and the stored
activations in bfloat16 and accumulates in FP32.  This oracle evaluates in
FP64 with bfloat16 rounding (round to nearest even) at the same points:
features, convolution weights, each stored convolution activation, and the
masked activation gradients fed to the weight and data products.  With
``bf16=False`` everything stays FP64 (for the finite-difference pins).
"""
from __future__ import annotations

import numpy as np

CELLS = 128
SHAPES = [("w1", (16, 3, 3, 3)), ("b1", (16,)), ("w2", (32, 16, 3, 3)), ("b2", (32,)),
          ("w3", (32, 32, 3, 3)), ("b3", (32,)), ("wf", (32,)), ("bf", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    x = np.asarray(x, dtype=np.float64)
    f = x.astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    # float64 -> float32 may round once already; bfloat16 of the float32 is
    # what the GPU stores when its FP32 value equals the float32 here
    return np.where(np.isfinite(x), out, x)


def unflatten(theta):
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def flatten(d):
    return np.concatenate([np.asarray(d[name], np.float64).ravel() for name, _ in SHAPES])


# --------------------------------------------------------------- features
def cell_index(n, cells=CELLS):
    """Cell of each of n positions: floor(i * cells / n)."""
    return (np.arange(n) * cells) // n


def features(img, Z1, Z2, bits, cells=CELLS):
    """3 x cells x cells: mean value / (2^bits - 1), non-zero fraction of Z1,
    of Z2, per cell of an area-downsample (empty cells give 0)."""
    H, W = img.shape
    cy, cx = cell_index(H, cells), cell_index(W, cells)
    flat = (cy[:, None] * cells + cx[None, :]).ravel()
    cnt = np.bincount(flat, minlength=cells * cells).astype(np.float64)
    f = np.zeros((3, cells * cells))
    f[0] = np.bincount(flat, weights=img.astype(np.float64).ravel(), minlength=cells * cells)
    f[1] = np.bincount(flat, weights=(Z1 != 0).ravel().astype(np.float64), minlength=cells * cells)
    f[2] = np.bincount(flat, weights=(Z2 != 0).ravel().astype(np.float64), minlength=cells * cells)
    with np.errstate(invalid="ignore", divide="ignore"):
        f = np.where(cnt > 0, f / np.maximum(cnt, 1), 0.0)
    f[0] /= float((1 << bits) - 1)
    return f.reshape(3, cells, cells)


# --------------------------------------------------------------- network
def conv_s2(x, w, b):
    """3x3 convolution (cross-correlation), stride 2, zero padding 1.
    x: (B, Ci, H, W), w: (Co, Ci, 3, 3) -> (B, Co, H/2, W/2)."""
    B, Ci, H, W = x.shape
    Co = w.shape[0]
    Ho, Wo = H // 2, W // 2
    xp = np.zeros((B, Ci, H + 2, W + 2))
    xp[:, :, 1:H + 1, 1:W + 1] = x
    out = np.zeros((B, Co, Ho, Wo))
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, :, ky:ky + 2 * Ho:2, kx:kx + 2 * Wo:2]        # (B, Ci, Ho, Wo)
            out += np.einsum("bchw,oc->bohw", patch, w[:, :, ky, kx], optimize=True)
    return out + b[None, :, None, None]


def conv_s2_backward(x, w, g):
    """Gradients of conv_s2 given g = dL/dout: (dx, dw, db)."""
    B, Ci, H, W = x.shape
    Ho, Wo = g.shape[2], g.shape[3]
    xp = np.zeros((B, Ci, H + 2, W + 2))
    xp[:, :, 1:H + 1, 1:W + 1] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, :, ky:ky + 2 * Ho:2, kx:kx + 2 * Wo:2]
            dw[:, :, ky, kx] = np.einsum("bohw,bchw->oc", g, patch, optimize=True)
            dxp[:, :, ky:ky + 2 * Ho:2, kx:kx + 2 * Wo:2] += np.einsum("bohw,oc->bchw", g, w[:, :, ky, kx],
                                                                      optimize=True)
    return dxp[:, :, 1:H + 1, 1:W + 1], dw, g.sum(axis=(0, 2, 3))


def forward(theta, feats, bf=True):
    """Returns (logits, cache).  feats: (B, 3, 128, 128)."""
    p = unflatten(theta)
    r = bf16 if bf else (lambda v: np.asarray(v, np.float64))
    x0 = r(feats)
    w = [r(p["w1"]), r(p["w2"]), r(p["w3"])]
    a1 = r(np.maximum(conv_s2(x0, w[0], p["b1"]), 0.0))
    a2 = r(np.maximum(conv_s2(a1, w[1], p["b2"]), 0.0))
    a3 = r(np.maximum(conv_s2(a2, w[2], p["b3"]), 0.0))
    gap = a3.mean(axis=(2, 3))                       # (B, 32)
    z = gap @ p["wf"] + p["bf"][0]
    return z, dict(x0=x0, a1=a1, a2=a2, a3=a3, gap=gap, w=w, p=p, bf=bf)


def bce(z, y):
    """Mean binary cross-entropy with logits."""
    return float(np.mean(np.maximum(z, 0) - z * y + np.log1p(np.exp(-np.abs(z)))))


def backward(theta, feats, labels, bf=True):
    """(loss, gradient of the mean loss w.r.t. theta)."""
    z, c = forward(theta, feats, bf)
    r = bf16 if bf else (lambda v: np.asarray(v, np.float64))
    y = np.asarray(labels, np.float64)
    B = z.shape[0]
    dz = (1.0 / (1.0 + np.exp(-z)) - y) / B          # (B,)
    p = c["p"]
    g = {"wf": c["gap"].T @ dz, "bf": np.array([dz.sum()])}
    dgap = dz[:, None] * p["wf"][None, :]            # (B, 32)
    da3 = np.broadcast_to(dgap[:, :, None, None] / 256.0, c["a3"].shape)
    g3 = r(da3 * (c["a3"] > 0))
    dx2, g["w3"], g["b3"] = conv_s2_backward(c["a2"], c["w"][2], g3)
    g2 = r(dx2 * (c["a2"] > 0))
    dx1, g["w2"], g["b2"] = conv_s2_backward(c["a1"], c["w"][1], g2)
    g1 = r(dx1 * (c["a1"] > 0))
    _, g["w1"], g["b1"] = conv_s2_backward(c["x0"], c["w"][0], g1)
    return bce(z, y), flatten(g)


def adamw(theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, wd=1e-4):
    """One AdamW step (decoupled weight decay on every parameter); returns
    (theta, m, v)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    theta = theta - lr * (mh / (np.sqrt(vh) + eps) + wd * theta)
    return theta, m, v


def init(seed):
    """He-uniform initialisation from a seed (FP32 values)."""
    rng = np.random.default_rng(seed)
    d = {}
    for name, shape in SHAPES:
        if name.startswith("w"):
            fan_in = int(np.prod(shape[1:])) if len(shape) > 1 else shape[0]
            lim = np.sqrt(6.0 / fan_in)
            d[name] = rng.uniform(-lim, lim, size=shape)
        else:
            d[name] = np.zeros(shape)
    return flatten(d).astype(np.float32).astype(np.float64)


# --------------------------------------------------------------- labels
def smoothing_label(E_noisy, F_noisy, E_clean):
    """The smoothing label of one tile (the reading of the labelling rule:
    the abstract and Sec. 4 let the noise in the extracted map decide the
    hybrid median of Sec. 3.4, and give no rule).

    E_noisy, F_noisy: the unsmoothed and smoothed maps of the noisy tile;
    E_clean: the unsmoothed map of its noise-free twin.  With N pixels,
    n_raw = #(E_noisy != E_clean) and n_med = #(F_noisy != E_clean), so
    D_raw = n_raw / N and D_med = n_med / N.  The median is worth applying
    when it lowers the disagreement by more than 1 % of itself: label 1 iff
    n_raw > 0 and D_med < 0.99 D_raw, decided exactly on the integers as
    100 n_med < 99 n_raw (a tile with D_raw = 0 gets 0).  The best-choice
    output of the tile is F_noisy for label 1, else E_noisy.

    Returns (d_raw, d_med, label, diff), diff = #(E_noisy != F_noisy): the
    pixels a wrong choice costs against the best-choice output."""
    E_noisy, F_noisy, E_clean = (np.asarray(a) for a in (E_noisy, F_noisy, E_clean))
    N = E_clean.size
    n_raw = int(np.count_nonzero(E_noisy != E_clean))
    n_med = int(np.count_nonzero(F_noisy != E_clean))
    label = int(n_raw > 0 and 100 * n_med < 99 * n_raw)
    return n_raw / N, n_med / N, label, int(np.count_nonzero(E_noisy != F_noisy))


def tile_label(noisy, clean, taps, **kw):
    """smoothing_label of a tile from its pixels and its noise-free twin's:
    the oracle pipeline (oracle.extract, with the masks taps and the
    parameters kw) on both, the noisy tile unsmoothed and smoothed, the
    twin unsmoothed."""
    import oracle
    o = oracle.extract(noisy, taps[0], taps[1], smooth=True, want_intermediates=True, **kw)
    c = oracle.extract(clean, taps[0], taps[1], smooth=False, **kw)
    return smoothing_label(o["E"], o["F"], c["F"])
