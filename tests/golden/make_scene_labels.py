"""Writes tests/golden/gate_labels_scenes.npz: the oracle's smoothing labels of
four-band scenes built like the 16384^2 benchmark workload (scenes.config5_*)
but smaller and from other seeds, cut into tiles -- training data of the
smoothing gate whose test is the benchmark scene itself (seed 5).
Calls only oracle/ and scenes; the labelling rule is
oracle.gate.smoothing_label (via oracle.gate.tile_label).

Per tile, as in make_gate_labels.py: D_raw = mean(E_noisy != E_clean),
D_med = mean(F_noisy != E_clean), label = [D_raw > 0 and D_med < 0.99 D_raw];
diff = pixels where E_noisy and F_noisy differ.  Columns scene_seed, band, ty,
tx locate the tile (scenes.config5_tile(config5_base(size, seed), band, ty,
tx, tile, seed)).

Run: python tests/golden/make_scene_labels.py [first_seed] [count] [size] [tile]
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
    first = int(sys.argv[1]) if len(sys.argv) > 1 else 1001
    count = int(sys.argv[2]) if len(sys.argv) > 2 else 10
    size = int(sys.argv[3]) if len(sys.argv) > 3 else 8192
    tile = int(sys.argv[4]) if len(sys.argv) > 4 else 2048
    taps = (oracle.log_mask(5, 0.8, 16)[0], oracle.log_mask(9, 1.4, 16)[0])
    rows = []
    t0 = time.time()
    for seed in range(first, first + count):
        base = scenes.config5_base(size, seed)
        for b, ty, tx in scenes.config5_index(size, tile):
            noisy, clean, sigma, density = scenes.config5_tile(base, b, ty, tx, tile, seed)
            d_raw, d_med, label, diff = gate.tile_label(noisy, clean, taps)
            rows.append((seed, b, ty, tx, d_raw, d_med, label, diff, sigma, density))
        print(f"scene {seed}: {len(rows)} tiles, {time.time() - t0:.0f} s", flush=True)
    a = np.array(rows, dtype=np.float64)
    np.savez_compressed(os.path.join(HERE, "gate_labels_scenes.npz"), scene_seed=a[:, 0].astype(np.int32),
                        band=a[:, 1].astype(np.int32), ty=a[:, 2].astype(np.int32), tx=a[:, 3].astype(np.int32),
                        d_raw=a[:, 4].astype(np.float32), d_med=a[:, 5].astype(np.float32),
                        label=a[:, 6].astype(np.uint8), diff=a[:, 7].astype(np.int64),
                        sigma=a[:, 8].astype(np.float32), density=a[:, 9].astype(np.float32),
                        scene_size=np.int32(size), tile=np.int32(tile), size=np.int32(tile),
                        count=np.int32(len(rows)))


if __name__ == "__main__":
    main()
