"""Writes tests/golden/config5_labels.npz: the oracle's best-choice labels of
the four-band 16384^2 workload cut into 2048^2 tiles (scenes.config5_*).
Calls only oracle/ and scenes; the labelling rule is
oracle.gate.smoothing_label (via oracle.gate.tile_label).

Per tile: E_noisy and F_noisy are the oracle's unsmoothed and hybrid-median
maps of the noisy tile, E_clean the unsmoothed map of the noise-free tile;
D_raw = mean(E_noisy != E_clean), D_med = mean(F_noisy != E_clean);
label = [D_raw > 0 and D_med < 0.99 D_raw] (the best choice is F_noisy when
the label is 1, else E_noisy); diff = number of pixels where E_noisy and
F_noisy differ (what a wrong choice costs in agreement with the best-choice
output); sha = SHA-256 of the noisy tile's bytes.

Run: python tests/golden/make_config5_labels.py [size] [tile]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from oracle import gate  # noqa: E402
from paper_1304_3992_amd import scenes  # noqa: E402


def main():
    size = int(sys.argv[1]) if len(sys.argv) > 1 else 16384
    tile = int(sys.argv[2]) if len(sys.argv) > 2 else 2048
    taps = (oracle.log_mask(5, 0.8, 16)[0], oracle.log_mask(9, 1.4, 16)[0])
    t0 = time.time()
    base = scenes.config5_base(size)
    print(f"base {time.time() - t0:.0f} s", flush=True)
    rows, shas = [], []
    index = scenes.config5_index(size, tile)
    for k, (b, ty, tx) in enumerate(index):
        noisy, clean, sigma, density = scenes.config5_tile(base, b, ty, tx, tile)
        d_raw, d_med, label, diff = gate.tile_label(noisy, clean, taps)
        rows.append((d_raw, d_med, label, diff, sigma, density))
        shas.append(scenes.sha256(noisy))
        if (k + 1) % 16 == 0:
            print(f"{k + 1}/{len(index)} tiles, {time.time() - t0:.0f} s", flush=True)
    a = np.array(rows, dtype=np.float64)
    np.savez_compressed(os.path.join(HERE, "config5_labels.npz"), d_raw=a[:, 0], d_med=a[:, 1],
                        label=a[:, 2].astype(np.uint8), diff=a[:, 3].astype(np.int64),
                        sigma=a[:, 4], density=a[:, 5], sha=np.array(shas), size=np.int32(size),
                        tile=np.int32(tile), base_sha=scenes.sha256(base))


if __name__ == "__main__":
    main()
