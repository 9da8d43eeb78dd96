"""What the trained gate gains, on tiles it was not trained on.

The committed parameters (paper_1304_3992_amd/gate_weights.bin, trained by
paper_1304_3992_amd/train_gate.py on the first 80 % of the 20 000 labelled
tiles) decide, on 300 tiles of the held-out last 10 %, whether to smooth.
The oracle scores the decisions: its labels (tests/golden/gate_labels.npz)
say which of the unsmoothed and smoothed maps is the best choice, and its
own maps of each tile say how many pixels the two differ in.  The gated
output must agree with the oracle's best-choice output on more pixels than
always smoothing and than never smoothing, and the gate must pick the best
choice on most tiles."""
import os

import numpy as np
import pytest

import oracle
from paper_1304_3992_amd import logfx, scenes
from parity import masks, to_device

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "paper_1304_3992_amd", "gate_weights.bin")
LABELS = os.path.join(ROOT, "tests", "golden", "gate_labels.npz")


def test_gate_agrees_with_best_choice_better_than_never_or_always():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    d = np.load(LABELS)
    count, size = int(d["count"]), int(d["size"])
    idx = np.arange(int(0.9 * count), int(0.9 * count) + 300)   # the test split
    orc_t, lib_t = masks()
    params = logfx.Params(*lib_t, smooth=logfx.SMOOTH_GATE)
    tiles = [scenes.gate_tile(int(i), size, twin=False)[0] for i in idx]
    with logfx.Context(0) as ctx:
        ctx.gate_load(WEIGHTS)
        z, _ = ctx.gate([to_device(t) for t in tiles], params, bits=11)
        dec = z.cpu().numpy() > 0
    diff = np.array([int((o["E"] != o["F"]).sum()) for o in
                     (oracle.extract(t, *orc_t, smooth=True, want_intermediates=True) for t in tiles)])
    lab = d["label"][idx] == 1
    px = float(len(idx) * size * size)

    def agreement(choice):
        return 1.0 - diff[choice != lab].sum() / px

    a_gate, a_always, a_never = agreement(dec), agreement(np.ones_like(lab)), agreement(np.zeros_like(lab))
    acc = float((dec == lab).mean())
    print(f"held-out: decision accuracy {acc:.3f}; agreement with the best choice: gated {a_gate:.5f}, "
          f"always {a_always:.5f}, never {a_never:.5f}")
    assert a_gate > a_always and a_gate > a_never
    assert acc > 0.85
