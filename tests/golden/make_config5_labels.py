"""Writes the oracle's records of the four-band 16384^2 workload cut into
2048^2 tiles (scenes.config5_*): tests/golden/config5_labels.npz (each
(band, tile) with its own noise level) and, with --per-band,
tests/golden/config5_perband_labels.npz (one noise level per band).
Calls only oracle/ and scenes; the labelling rule is
oracle.gate.smoothing_label.

Per tile: E_noisy and F_noisy are the oracle's unsmoothed and hybrid-median
maps of the noisy tile, E_clean the unsmoothed map of the noise-free tile;
D_raw = mean(E_noisy != E_clean), D_med = mean(F_noisy != E_clean);
label = [D_raw > 0 and D_med < 0.99 D_raw] (the best choice is F_noisy when
the label is 1, else E_noisy); diff = number of pixels where E_noisy and
F_noisy differ (what a wrong choice costs in agreement with the best-choice
output); sha = SHA-256 of the noisy tile's bytes; sha_E / sha_F = SHA-256
of the oracle's E_noisy / F_noisy bytes (0/1 uint8, row-major); logit = the
oracle network (oracle.gate.forward, bfloat16 rounding points) on the
oracle features of the noisy tile with the parameters of
paper_1304_3992_amd/gate_weights.bin, whose SHA-256 is weights_sha.

Run: python tests/golden/make_config5_labels.py [--per-band] [size] [tile]
"""
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import gate  # noqa: E402
from paper_1304_3992_amd import scenes  # noqa: E402

WEIGHTS = os.path.join(ROOT, "paper_1304_3992_amd", "gate_weights.bin")
_BASE = None
_ARGS = None


def read_weights(path):
    """The parameters of a LOGFXGT1 file: 8-byte tag, int32 count, int32 0,
    then the FP32 values (little-endian)."""
    raw = open(path, "rb").read()
    assert raw[:8] == b"LOGFXGT1"
    n, z = np.frombuffer(raw[8:16], "<i4")
    assert n == gate.NPARAM and z == 0 and len(raw) == 16 + 4 * n
    return np.frombuffer(raw[16:], "<f4").astype(np.float64)


def one_tile(job):
    b, ty, tx = job
    size, tile, per_band, theta = _ARGS
    taps = (oracle.log_mask(5, 0.8, 16)[0], oracle.log_mask(9, 1.4, 16)[0])
    noisy, clean, sigma, density = scenes.config5_tile(_BASE, b, ty, tx, tile, per_band=per_band)
    o = oracle.extract(noisy, taps[0], taps[1], smooth=True, want_intermediates=True, nthreads=1)
    c = oracle.extract(clean, taps[0], taps[1], smooth=False, nthreads=1)
    d_raw, d_med, label, diff = gate.smoothing_label(o["E"], o["F"], c["F"])
    f = gate.features(noisy, o["Z1"], o["Z2"], 11)
    z = float(gate.forward(theta, f[None])[0][0])
    return ((d_raw, d_med, label, diff, sigma, density, z),
            (scenes.sha256(noisy), scenes.sha256(o["E"]), scenes.sha256(o["F"])))


def main():
    global _BASE, _ARGS
    argv = [a for a in sys.argv[1:] if a != "--per-band"]
    per_band = "--per-band" in sys.argv[1:]
    size = int(argv[0]) if len(argv) > 0 else 16384
    tile = int(argv[1]) if len(argv) > 1 else 2048
    theta = read_weights(WEIGHTS)
    t0 = time.time()
    _BASE = scenes.config5_base(size)
    base_sha = scenes.sha256(_BASE)
    print(f"base {time.time() - t0:.0f} s", flush=True)
    _ARGS = (size, tile, per_band, theta)
    index = scenes.config5_index(size, tile)
    with mp.get_context("fork").Pool(min(16, os.cpu_count() or 1)) as pool:
        res = []
        for k, r in enumerate(pool.imap(one_tile, index, chunksize=2)):
            res.append(r)
            if (k + 1) % 32 == 0:
                print(f"{k + 1}/{len(index)} tiles, {time.time() - t0:.0f} s", flush=True)
    a = np.array([r[0] for r in res], dtype=np.float64)
    shas = np.array([r[1] for r in res])
    name = "config5_perband_labels.npz" if per_band else "config5_labels.npz"
    np.savez_compressed(os.path.join(HERE, name), d_raw=a[:, 0], d_med=a[:, 1],
                        label=a[:, 2].astype(np.uint8), diff=a[:, 3].astype(np.int64),
                        sigma=a[:, 4], density=a[:, 5], logit=a[:, 6], sha=shas[:, 0], sha_E=shas[:, 1],
                        sha_F=shas[:, 2], size=np.int32(size), tile=np.int32(tile), base_sha=base_sha,
                        weights_sha=scenes.sha256(np.frombuffer(open(WEIGHTS, "rb").read(), np.uint8)),
                        per_band=np.int32(per_band))


if __name__ == "__main__":
    main()
