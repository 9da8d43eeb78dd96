"""Pins of the smoothing-label rule (oracle.gate.smoothing_label /
tile_label), which writes every stored gate label and the best-choice output
the four-band benchmark is scored against (no GPU).

The rule reads the abstract and Sec. 4 (the noise in the extracted map
decides the median): label 1 iff the median lowers the tile's disagreement
with its noise-free twin's unsmoothed map by more than 1 % of itself.  The
pins below are chosen so that each plausible slip fails one of them:
'<=' for '<' (the exact 1 % boundary), an absolute 1 % in place of a
relative one, a smoothed twin map (a tile identical to its twin), a missing
D_raw = 0 guard; and every stored file is re-derived from the rule."""
import os

import numpy as np
import pytest

import oracle
from oracle import gate
from paper_1304_3992_amd import scenes

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _maps(N, n_raw, n_med, seed=0):
    """Maps of N pixels: E_clean random, E_noisy differing from it at n_raw
    pixels, F_noisy at n_med pixels (disjoint choices)."""
    rng = np.random.default_rng(seed)
    clean = rng.integers(0, 2, N).astype(np.uint8)
    order = rng.permutation(N)
    E = clean.copy()
    E[order[:n_raw]] ^= 1
    F = clean.copy()
    F[order[n_raw:n_raw + n_med]] ^= 1
    return E, F, clean


def test_identical_maps_give_zero_and_label_0():
    m = np.zeros((8, 8), np.uint8)
    assert gate.smoothing_label(m, m, m) == (0.0, 0.0, 0, 0)
    # D_raw = 0 with a worse smoothed map: still 0 (no division, no gain)
    F = m.copy()
    F[3, 3] = 1
    assert gate.smoothing_label(m, F, m)[2] == 0


def test_exact_one_percent_boundary_is_not_a_gain():
    # n_raw = 100, n_med = 99: D_med = 0.99 D_raw exactly -> 0 ('<=' would say 1)
    E, F, C = _maps(10000, 100, 99)
    d_raw, d_med, label, _ = gate.smoothing_label(E, F, C)
    assert (d_raw, d_med, label) == (0.01, 0.0099, 0)
    # one pixel better -> 1
    E, F, C = _maps(10000, 100, 98)
    assert gate.smoothing_label(E, F, C)[2] == 1
    # the same boundary at a count where 0.99 n_raw is not an integer
    assert gate.smoothing_label(*_maps(20000, 150, 148))[2] == 1    # 148 < 148.5
    assert gate.smoothing_label(*_maps(20000, 150, 149))[2] == 0


def test_relative_not_absolute():
    # D_raw 0.10 -> D_med 0.095: a 5 % relative gain (label 1) that an
    # absolute 1-point rule (0.005 < 0.01) would reject
    assert gate.smoothing_label(*_maps(10000, 1000, 950))[2] == 1
    # D_raw 0.5 -> D_med 0.4955: 0.9 % relative (label 0) although the
    # absolute drop, 0.0045, is what a rule on a 0.5 % scale would accept
    assert gate.smoothing_label(*_maps(20000, 10000, 9910))[2] == 0
    # a worse median is never chosen
    assert gate.smoothing_label(*_maps(10000, 100, 150))[2] == 0


def test_diff_counts_unsmoothed_against_smoothed():
    E, F, C = _maps(5000, 40, 30, seed=3)
    # E and F differ where exactly one of them differs from C (disjoint sets)
    assert gate.smoothing_label(E, F, C)[3] == 70


def test_tile_equal_to_its_twin():
    """A tile with no noise: its unsmoothed map equals its twin's, so D_raw
    = 0 and the label is 0, and D_med counts where the median changes the
    map.  A smoothed twin map would give D_med = 0 < D_raw and label 1."""
    img = scenes.config1()[:256, :256]
    taps = (oracle.log_mask(5, 0.8, 16)[0], oracle.log_mask(9, 1.4, 16)[0])
    d_raw, d_med, label, diff = gate.tile_label(img, img, taps)
    assert d_raw == 0.0 and label == 0
    assert diff > 0 and d_med * img.size == diff


def _rule_from_fractions(d_raw, d_med, N):
    # the stored fractions are n / N with N a power of two, exact in float32
    n_raw = np.rint(np.asarray(d_raw, np.float64) * N).astype(np.int64)
    n_med = np.rint(np.asarray(d_med, np.float64) * N).astype(np.int64)
    assert np.array_equal(n_raw.astype(np.float64) / N, np.asarray(d_raw, np.float64))
    assert np.array_equal(n_med.astype(np.float64) / N, np.asarray(d_med, np.float64))
    return ((n_raw > 0) & (100 * n_med < 99 * n_raw)).astype(np.uint8)


@pytest.mark.parametrize("name", ["gate_labels.npz", "gate_labels_2048.npz", "gate_labels_1024b.npz",
                                  "gate_labels_scenes.npz", "config5_labels.npz",
                                  "config5_perband_labels.npz"])
def test_every_stored_label_follows_the_rule(name):
    d = np.load(os.path.join(GOLDEN, name))
    side = int(d["tile"]) if "tile" in d.files else int(d["size"])
    assert side & (side - 1) == 0
    assert np.array_equal(d["label"], _rule_from_fractions(d["d_raw"], d["d_med"], side * side)), name


def _check_row(d, i, res, fields=("d_raw", "d_med", "label")):
    got = dict(zip(("d_raw", "d_med", "label", "diff"), res))
    for k in fields:
        assert np.float64(d[k][i]) == np.float64(np.asarray(got[k], d[k].dtype)), (k, i, d[k][i], got[k])


@pytest.mark.parametrize("name,count,size,seed,band", [
    ("gate_labels.npz", 20000, 512, 400000, False),
    ("gate_labels_2048.npz", 2000, 2048, 600000, False),
    ("gate_labels_1024b.npz", 4000, 1024, 700000, True)])
def test_stored_training_labels_recomputed(name, count, size, seed, band):
    """A spread of tiles of each training file regenerated from its seed and
    labelled again by the oracle: the stored fractions and labels return."""
    d = np.load(os.path.join(GOLDEN, name))
    assert int(d["count"]) == count and int(d["size"]) == size
    if "base_seed" in d.files:
        assert int(d["base_seed"]) == seed
    if "band" in d.files:
        assert bool(int(d["band"])) == band
    taps = (oracle.log_mask(5, 0.8, 16)[0], oracle.log_mask(9, 1.4, 16)[0])
    picks = np.linspace(0, count - 1, 6 if size <= 1024 else 3).astype(int)
    picks = sorted(set(picks.tolist()) | {int(np.argmax(d["label"])), int(np.argmin(d["label"]))})
    for i in picks:
        noisy, clean, sigma, density = scenes.gate_tile(i, size, seed, band=band)
        assert np.float32(sigma) == d["sigma"][i] and np.float32(density) == d["density"][i]
        _check_row(d, i, gate.tile_label(noisy, clean, taps))


def test_stored_scene_labels_recomputed():
    d = np.load(os.path.join(GOLDEN, "gate_labels_scenes.npz"))
    size, tile = int(d["scene_size"]), int(d["tile"])
    taps = (oracle.log_mask(5, 0.8, 16)[0], oracle.log_mask(9, 1.4, 16)[0])
    seed = int(d["scene_seed"][0])
    base = scenes.config5_base(size, seed)
    rows = np.flatnonzero(d["scene_seed"] == seed)
    for i in rows[np.linspace(0, len(rows) - 1, 4).astype(int)]:
        noisy, clean, _, _ = scenes.config5_tile(base, int(d["band"][i]), int(d["ty"][i]), int(d["tx"][i]), tile,
                                                 seed)
        _check_row(d, i, gate.tile_label(noisy, clean, taps), ("d_raw", "d_med", "label", "diff"))


@pytest.fixture(scope="module")
def config5_base():
    return scenes.config5_base()


@pytest.mark.parametrize("name,per_band", [("config5_labels.npz", False), ("config5_perband_labels.npz", True)])
def test_config5_labels_recomputed_and_inputs_unchanged(config5_base, name, per_band):
    """The four-band benchmark's best-choice records (per-tile and per-band
    noise): the generated base scene and tiles still hash to the stored
    values (so the stored records belong to the tiles the benchmark runs),
    and tiles relabelled by the oracle give the stored fractions, labels,
    E/F difference counts, map hashes and network logits."""
    d = np.load(os.path.join(GOLDEN, name))
    assert scenes.sha256(config5_base) == str(d["base_sha"])
    assert bool(int(d["per_band"])) == per_band
    weights = os.path.join(os.path.dirname(GOLDEN), "..", "paper_1304_3992_amd", "gate_weights.bin")
    raw = open(weights, "rb").read()
    assert scenes.sha256(np.frombuffer(raw, np.uint8)) == str(d["weights_sha"])
    theta = np.frombuffer(raw[16:], "<f4").astype(np.float64)
    index = scenes.config5_index()
    assert len(index) == len(d["label"])
    taps = (oracle.log_mask(5, 0.8, 16)[0], oracle.log_mask(9, 1.4, 16)[0])
    picks = sorted({0, len(index) - 1, int(np.argmax(d["label"])), int(np.argmin(d["label"])), 77, 150})
    for i in picks:
        b, ty, tx = index[i]
        noisy, clean, sigma, _ = scenes.config5_tile(config5_base, b, ty, tx, per_band=per_band)
        assert scenes.sha256(noisy) == str(d["sha"][i])
        assert np.float64(sigma) == d["sigma"][i]
        o = oracle.extract(noisy, taps[0], taps[1], smooth=True, want_intermediates=True)
        c = oracle.extract(clean, taps[0], taps[1], smooth=False)
        _check_row(d, i, gate.smoothing_label(o["E"], o["F"], c["F"]), ("d_raw", "d_med", "label", "diff"))
        assert scenes.sha256(o["E"]) == str(d["sha_E"][i]) and scenes.sha256(o["F"]) == str(d["sha_F"][i])
        z = gate.forward(theta, gate.features(noisy, o["Z1"], o["Z2"], 11)[None])[0][0]
        assert float(z) == float(d["logit"][i])
