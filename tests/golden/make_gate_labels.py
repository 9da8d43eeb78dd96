"""Writes tests/golden/gate_labels.npz: the oracle's smoothing labels of the
gate's training tiles (scenes.gate_tile).  Calls only oracle/ and scenes; the labelling rule is
oracle.gate.smoothing_label (via oracle.gate.tile_label).

Per tile (the reading of the benchmark's labelling rule): E_noisy and
F_noisy are the oracle's unsmoothed and hybrid-median maps of the noisy tile,
E_clean the unsmoothed map of its noise-free twin;
D_raw = mean(E_noisy != E_clean), D_med = mean(F_noisy != E_clean), and the
label is 1 when the median reduces the disagreement by more than 1 %
(relative): D_med < 0.99 D_raw.  D_raw = 0 gives label 0.

Run: python tests/golden/make_gate_labels.py [count] [size] [base_seed] [band]
(size 512 writes gate_labels.npz, other sizes gate_labels_<size>.npz; with
band = 1 the tiles are mapped to random bands first, scenes.gate_tile(band=True),
and the file is gate_labels_<size>b.npz)
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


def label_tile(i, size, taps, base_seed, band):
    noisy, clean, sigma, density = scenes.gate_tile(i, size, base_seed, band=band)
    d_raw, d_med, label, _ = gate.tile_label(noisy, clean, taps)
    return d_raw, d_med, label, sigma, density


def main():
    count = int(sys.argv[1]) if len(sys.argv) > 1 else 20000
    size = int(sys.argv[2]) if len(sys.argv) > 2 else 512
    base_seed = int(sys.argv[3]) if len(sys.argv) > 3 else 400000
    band = len(sys.argv) > 4 and sys.argv[4] == "1"
    taps = (oracle.log_mask(5, 0.8, 16)[0], oracle.log_mask(9, 1.4, 16)[0])
    rows = []
    t0 = time.time()
    for i in range(count):
        rows.append(label_tile(i, size, taps, base_seed, band))
        if (i + 1) % 500 == 0:
            print(f"{i + 1}/{count} tiles, {time.time() - t0:.0f} s", flush=True)
    a = np.array(rows, dtype=np.float64)
    name = "gate_labels.npz" if size == 512 and not band else f"gate_labels_{size}{'b' if band else ''}.npz"
    np.savez_compressed(os.path.join(HERE, name), d_raw=a[:, 0].astype(np.float32),
                        d_med=a[:, 1].astype(np.float32), label=a[:, 2].astype(np.uint8),
                        sigma=a[:, 3].astype(np.float32), density=a[:, 4].astype(np.float32),
                        size=np.int32(size), count=np.int32(count), base_seed=np.int32(base_seed),
                        band=np.int32(band))


if __name__ == "__main__":
    main()
