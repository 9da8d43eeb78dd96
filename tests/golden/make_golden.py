"""Writes tests/golden/masks.json from the oracle alone.

The file freezes the integer taps of the zero-sum LoG masks (eq. (1),
Sec. 3.1, sampled, mean-removed and snapped to a power-of-two grid) used by
the benchmark workloads, so that any later change to the mask construction
shows up as a test failure and has to be justified.
Run: python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402

CASES = [(5, 0.8, 16), (9, 1.4, 16), (5, 0.8, 23), (9, 1.4, 23), (3, 0.5, 16), (7, 1.0, 16)]


def main():
    out = []
    for size, sigma, bits in CASES:
        taps, u = oracle.log_mask(size, sigma, bits)
        k = (taps.astype("float64") / u).round().astype(int)
        out.append({"size": size, "sigma": sigma, "grid_bits": bits, "unit": u,
                    "k": k.tolist()})
    with open(os.path.join(HERE, "masks.json"), "w") as f:
        json.dump({"source": "oracle.log_mask (eq. (1), Sec. 3.1)", "masks": out}, f, indent=1)


if __name__ == "__main__":
    main()
