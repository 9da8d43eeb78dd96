"""GPU parity of the smoothing gate against its FP64 oracle (oracle/gate.py):
features gathered by pass 1, the network's logits, its gradients, the AdamW
step, training, and the gated pipeline.

Tolerances.  Features are exact cell sums on both sides, divided in the same
order in FP64 and rounded once to bfloat16: bit-equal.  The network
accumulates in FP32 on the matrix cores where the oracle uses FP64, and both
round every stored activation to bfloat16; a value within ~1e-6 relative of
a bfloat16 rounding boundary may round the other way (one bfloat16 step,
2^-8 relative, on about 3 in 10^4 values).  Averaged by the pooling this
moves a logit by ~1e-4 at most in these cases: logits must agree within
1e-3 (relative, with 1e-3 absolute floor), and a decision may differ only
where |logit| < 1e-3.  Gradients see the flips directly (they are not
averaged before the weight products): per parameter tensor the relative L2
error must stay below 1e-2.  The AdamW step is FP32 against FP64 on the
same gradient: 1e-5 relative."""
import os

import numpy as np
import pytest

import oracle
from oracle import gate as og
from paper_1304_3992_amd import logfx, scenes
from parity import masks, run_oracle, to_device

pytestmark = pytest.mark.gpu

LOGIT_TOL = 1e-3
GRAD_REL_L2 = 1e-2


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    c = logfx.Context(0)
    yield c
    c.close()


def _bf16_dev(x):
    """Seeded FP64 values to a device bfloat16 tensor (round to nearest even)."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, np.float32)).to(torch.bfloat16).cuda()


def _features_cases():
    rng = np.random.default_rng(71)
    return [
        ("scene_u11_512", scenes.gate_tile(3)[0], 11),
        ("scene_u11_ragged", scenes.panchromatic(301, 517, 72, n_rect=60, n_poly=4, noise_sigma=9.0,
                                                 sp_density=0.03, bits=11), 11),
        ("u8_small", rng.integers(0, 256, (100, 77)).astype(np.uint8), 8),
        ("u8_tall", scenes.config1()[:, :40], 8),
        ("u16_fp64", rng.integers(0, 65536, (150, 260)).astype(np.uint16), 16),
        ("one_pixel", np.array([[9]], np.uint8), 8),
    ]


@pytest.mark.parametrize("case", range(6))
def test_features_bit_exact(ctx, case):
    """Pass-1 cell sums -> bfloat16 features equal the oracle's features of
    the oracle's crossing maps, value for value (single-image calls)."""
    import torch
    name, img, bits = _features_cases()[case]
    orc_t, lib_t = masks()
    params = logfx.Params(*lib_t)
    f = ctx.gate_features(to_device(img), params, bits=bits)
    torch.cuda.synchronize()
    got = f.float().cpu().numpy().astype(np.float64)[0]
    o = run_oracle(img, orc_t)
    ref = og.bf16(og.features(img, o["Z1"], o["Z2"], bits))
    bad = np.argwhere(got != ref)
    assert bad.size == 0, (name, bad[:5], got[tuple(bad[0])], ref[tuple(bad[0])])


def test_features_batch_equals_singles(ctx):
    """A batch of uneven tiles (several pass-1 tiles per image, several
    images per launch) gives each image its single-call features."""
    import torch
    tiles = scenes.config3(n=7, seed=73, base_seed=7300, lo=60, hi=900)
    _, lib_t = masks()
    params = logfx.Params(*lib_t)
    devs = [to_device(t) for t in tiles]
    fb = ctx.gate_features(devs, params, bits=8)
    singles = [ctx.gate_features(d, params, bits=8) for d in devs]
    torch.cuda.synchronize()
    for i, s in enumerate(singles):
        assert torch.equal(fb[i], s[0]), i


def _net_inputs(B, seed):
    rng = np.random.default_rng(seed)
    feats = rng.random((B, 3, 128, 128))
    feats[:, 1:] *= 0.6
    theta = og.init(seed)
    labels = (rng.random(B) < 0.5).astype(np.float64)
    return feats, theta, labels


@pytest.mark.parametrize("B,seed", [(1, 81), (5, 82), (19, 83)])
def test_forward_logits(ctx, B, seed):
    import torch
    feats, theta, _ = _net_inputs(B, seed)
    ctx.gate_set_params(theta)
    z = ctx.gate_forward(_bf16_dev(feats)).cpu().numpy().astype(np.float64)
    z_ref, _ = og.forward(theta, feats)
    np.testing.assert_allclose(z, z_ref, rtol=LOGIT_TOL, atol=LOGIT_TOL)


def test_forward_through_sample_indices(ctx):
    import torch
    feats, theta, _ = _net_inputs(12, 84)
    ctx.gate_set_params(theta)
    idx = torch.tensor([7, 0, 11, 7, 3], dtype=torch.int32, device="cuda")
    z = ctx.gate_forward(_bf16_dev(feats), idx).cpu().numpy().astype(np.float64)
    z_ref, _ = og.forward(theta, feats[[7, 0, 11, 7, 3]])
    np.testing.assert_allclose(z, z_ref, rtol=LOGIT_TOL, atol=LOGIT_TOL)


@pytest.mark.parametrize("B,seed", [(2, 91), (9, 92)])
def test_gradient_matches_oracle(ctx, B, seed):
    import torch
    feats, theta, labels = _net_inputs(B, seed)
    theta[og.NPARAM - 1] = 0.3
    ctx.gate_set_params(theta)
    lab = torch.tensor(labels, dtype=torch.float32, device="cuda")
    g, loss = ctx.gate_backward(_bf16_dev(feats), lab)
    g = g.cpu().numpy().astype(np.float64)
    loss_ref, g_ref = og.backward(theta, feats, labels)
    assert float(loss.cpu()[0]) == pytest.approx(loss_ref, rel=1e-4, abs=1e-5)
    o = 0
    for name, shape in og.SHAPES:
        n = int(np.prod(shape))
        a, r = g[o:o + n], g_ref[o:o + n]
        err = np.linalg.norm(a - r) / max(np.linalg.norm(r), 1e-30)
        assert err < GRAD_REL_L2, (name, err)
        o += n


def test_adamw_step_matches_oracle(ctx):
    """Three AdamW steps on given gradients: FP32 on the GPU, FP64 in the
    oracle, same formula."""
    import torch
    rng = np.random.default_rng(95)
    theta = og.init(95)
    ctx.gate_set_params(theta)
    m = np.zeros(og.NPARAM)
    v = np.zeros(og.NPARAM)
    th = theta.copy()
    for step in range(1, 4):
        gr = rng.normal(0, 1e-2, og.NPARAM).astype(np.float32).astype(np.float64)
        ctx.gate_step(3e-3, torch.tensor(gr, dtype=torch.float32, device="cuda"))
        th, m, v = og.adamw(th, gr, m, v, step, 3e-3)
    got = ctx.gate_get_params().astype(np.float64)
    np.testing.assert_allclose(got, th, rtol=1e-5, atol=1e-7)
    # the step also refreshed the forward kernels' copy of the weights: the
    # logits follow the stepped parameters
    feats, _, _ = _net_inputs(6, 96)
    z = ctx.gate_forward(_bf16_dev(feats)).cpu().numpy().astype(np.float64)
    z_ref, _ = og.forward(got, feats)
    np.testing.assert_allclose(z, z_ref, rtol=LOGIT_TOL, atol=LOGIT_TOL)


def test_parameters_round_trip_file(ctx, tmp_path):
    theta = og.init(96).astype(np.float32)
    ctx.gate_set_params(theta)
    p = str(tmp_path / "gate.bin")
    ctx.gate_save(p)
    with logfx.Context(0) as c2:
        c2.gate_load(p)
        assert np.array_equal(c2.gate_get_params(), theta)
    with open(p, "r+b") as f:
        f.write(b"XXXX")
    with logfx.Context(0) as c3:
        with pytest.raises(logfx.LogfxError) as e:
            c3.gate_load(p)
        assert e.value.code == logfx.EINVAL


def test_training_state_resumes_exactly(ctx, tmp_path):
    """Training stopped after some steps, saved with its AdamW moments and
    step count, and resumed in a fresh context ends with the same
    parameters, bit for bit, as the uninterrupted run; a corrupted or
    truncated state file is refused with the context left as it was."""
    import torch
    rng = np.random.default_rng(191)
    N = 96
    feats = rng.random((N, 3, 128, 128)) * 0.3
    y = rng.random(N) < 0.5
    feats[y, 2] += 0.4
    fd = _bf16_dev(feats)
    lab = torch.tensor(y.astype(np.float32), device="cuda")
    theta0 = og.init(192)

    def steps(c, it0, it1):
        g = torch.empty(og.NPARAM, dtype=torch.float32, device="cuda")
        for it in range(it0, it1):
            idx = torch.from_numpy(np.random.default_rng(500 + it).choice(N, 32, replace=False)
                                   .astype(np.int32)).cuda()
            c.gate_backward(fd, lab, idx, grad=g)
            c.gate_step(2e-3, g)

    ctx.gate_set_params(theta0)
    steps(ctx, 0, 12)
    whole = ctx.gate_get_params()
    ctx.gate_set_params(theta0)
    steps(ctx, 0, 7)
    path = str(tmp_path / "state.bin")
    ctx.gate_save_state(path)
    with logfx.Context(0) as c2:
        c2.gate_load_state(path)
        steps(c2, 7, 12)
        resumed = c2.gate_get_params()
    assert np.array_equal(resumed, whole)
    # the parameters alone (gate_load of the state file) restart the moments
    with logfx.Context(0) as c3:
        c3.gate_load(path)
        steps(c3, 7, 12)
        assert not np.array_equal(c3.gate_get_params(), whole)
    raw = open(path, "rb").read()
    before = ctx.gate_get_params()
    for bad in (raw[:-1], raw[:100] + bytes([raw[100] ^ 1]) + raw[101:], b"LOGFXGT1" + raw[8:]):
        with open(path, "wb") as f:
            f.write(bad)
        with pytest.raises(logfx.LogfxError) as e:
            ctx.gate_load_state(path)
        assert e.value.code == logfx.EINVAL
        assert np.array_equal(ctx.gate_get_params(), before)


def test_missing_gate_file_falls_back_to_always(ctx, tmp_path):
    """A missing or corrupt gate file leaves a fresh context without
    parameters: SMOOTH_GATE then runs as ALWAYS and the report says so."""
    import torch
    img = scenes.gate_tile(11)[0]
    _, lib_t = masks()
    with logfx.Context(0) as c:
        with pytest.raises(logfx.LogfxError):
            c.gate_load(str(tmp_path / "absent.bin"))
        bad = tmp_path / "bad.bin"
        bad.write_bytes(b"LOGFXGT1" + b"\x00" * 7)
        with pytest.raises(logfx.LogfxError):
            c.gate_load(str(bad))
        d = to_device(img)
        out, rep = c.extract(d, logfx.Params(*lib_t, smooth=logfx.SMOOTH_GATE), bits=11, report=True)
        ref = c.extract(d, logfx.Params(*lib_t, smooth=logfx.SMOOTH_ALWAYS), bits=11)
        torch.cuda.synchronize()
        assert rep["gate_fallback"] == 1 and rep["gated"] == 0 and rep["smoothed"] == 1
        assert torch.equal(out, ref)


def test_training_reduces_loss_deterministically(ctx):
    """Steps of backward + AdamW on a separable synthetic task: the loss
    falls, the accuracy rises, and two runs from the same start give the
    same parameters bit for bit (fixed-order reductions)."""
    import torch
    rng = np.random.default_rng(97)
    N = 256
    feats = rng.random((N, 3, 128, 128)) * 0.2
    y = (rng.random(N) < 0.5)
    feats[y, 1] += 0.5            # the positives have dense mask-1 crossings
    fd = _bf16_dev(feats)
    lab = torch.tensor(y.astype(np.float32), device="cuda")
    theta0 = og.init(98)

    def train():
        ctx.gate_set_params(theta0)
        losses = []
        g = torch.empty(og.NPARAM, dtype=torch.float32, device="cuda")
        for it in range(40):
            idx = torch.from_numpy(np.random.default_rng(it).choice(N, 64, replace=False).astype(np.int32)).cuda()
            _, loss = ctx.gate_backward(fd, lab, idx, grad=g)
            ctx.gate_step(3e-3, g)
            losses.append(float(loss.cpu()[0]))
        return losses, ctx.gate_get_params()

    l1, p1 = train()
    l2, p2 = train()
    assert np.array_equal(p1, p2)
    assert l1 == l2
    assert np.mean(l1[-5:]) < 0.5 * np.mean(l1[:5]), l1
    z = ctx.gate_forward(fd).cpu().numpy()
    assert ((z > 0) == y).mean() > 0.95


def _gate_tiles():
    out = []
    for i in range(6):
        noisy, _, _, _ = scenes.gate_tile(10_000 + i, size=256 + 64 * i)
        out.append(noisy)
    return out


def test_gated_pipeline_against_oracle_chain(ctx):
    """SMOOTH_GATE on a batch: every image's decision equals the oracle
    chain's (oracle maps -> oracle features -> oracle network) unless its
    logit lies within the tolerance of 0, and its output equals the
    oracle's smoothed or unsmoothed map accordingly (band rule)."""
    import torch
    from parity import compare
    tiles = _gate_tiles()
    orc_t, lib_t = masks()
    theta = og.init(99)
    theta[og.NPARAM - 1] = 0.0
    ctx.gate_set_params(theta)
    params = logfx.Params(*lib_t, smooth=logfx.SMOOTH_GATE)
    devs = [to_device(t) for t in tiles]
    outs, reps = ctx.extract_batch(devs, params, bits=11, report=True)
    logits, dec = ctx.gate(devs, params, bits=11)
    torch.cuda.synchronize()
    logits = logits.cpu().numpy()
    dec = dec.cpu().numpy()
    feats = []
    orcs = []
    for t in tiles:
        o = run_oracle(t, orc_t, smooth=True)
        orcs.append(o)
        feats.append(og.features(t, o["Z1"], o["Z2"], 11))
    z_ref, _ = og.forward(theta, np.stack(feats))
    for i, t in enumerate(tiles):
        r = reps[i]
        assert r["gated"] == 1 and r["gate_fallback"] == 0
        assert r["gate_logit"] == pytest.approx(float(logits[i]), abs=0)
        assert abs(logits[i] - z_ref[i]) <= LOGIT_TOL * (1 + abs(z_ref[i])), (i, logits[i], z_ref[i])
        if abs(z_ref[i]) > LOGIT_TOL:
            assert r["smoothed"] == int(z_ref[i] > 0), i
        assert dec[i] == r["smoothed"]
        o = orcs[i]
        ref = o if r["smoothed"] else {**o, "F": o["E"]}
        compare(outs[i].cpu().numpy(), ref, smooth=bool(r["smoothed"]))


def test_gate_bias_forces_each_choice_and_fallback(ctx):
    """With a large positive (negative) output bias every image is smoothed
    (not smoothed): the gated batch equals the ALWAYS (NEVER) batch bit for
    bit.  With no parameters in a context GATE falls back to ALWAYS and
    reports it."""
    import torch
    tiles = _gate_tiles()[:4]
    _, lib_t = masks()
    devs = [to_device(t) for t in tiles]
    always = ctx.extract_batch(devs, logfx.Params(*lib_t, smooth=True), bits=11)
    never = ctx.extract_batch(devs, logfx.Params(*lib_t, smooth=False), bits=11)
    gparams = logfx.Params(*lib_t, smooth=logfx.SMOOTH_GATE)
    theta = og.init(100)
    for bias, ref, flag in ((50.0, always, 1), (-50.0, never, 0)):
        theta[og.NPARAM - 1] = bias
        ctx.gate_set_params(theta)
        for graph in (1, 0):
            ctx.set_option(logfx.OPT_GRAPH, graph)
            outs, reps = ctx.extract_batch(devs, gparams, bits=11, report=True)
            torch.cuda.synchronize()
            for o, r, e in zip(outs, reps, ref):
                assert torch.equal(o, e)
                assert r["smoothed"] == flag and r["gated"] == 1
        ctx.set_option(logfx.OPT_GRAPH, 1)
        single, rep = ctx.extract(devs[0], gparams, bits=11, report=True)
        assert torch.equal(single, ref[0]) and rep["smoothed"] == flag
    with logfx.Context(0) as fresh:
        outs, reps = fresh.extract_batch(devs, gparams, bits=11, report=True)
        torch.cuda.synchronize()
        for o, r, e in zip(outs, reps, always):
            assert torch.equal(o, e)
            assert r["gate_fallback"] == 1 and r["gated"] == 0 and r["smoothed"] == 1
        with pytest.raises(logfx.LogfxError) as e:
            fresh.gate(devs, gparams, bits=11)
        assert e.value.code == logfx.EINVAL


@pytest.mark.parametrize("median_size", [3, 5])
def test_gated_batch_same_with_stored_or_recomputed_strengths(ctx, median_size):
    """The gated batch gives the same bytes and decisions whether pass 2
    reads the stored strengths or recomputes them, for both median sizes,
    and each image's output is its single-call output with that decision."""
    import torch
    tiles = _gate_tiles()[:5]
    _, lib_t = masks()
    theta = og.init(101)
    theta[og.NPARAM - 1] = 0.0
    ctx.gate_set_params(theta)
    params = logfx.Params(*lib_t, smooth=logfx.SMOOTH_GATE, median_size=median_size)
    devs = [to_device(t) for t in tiles]
    res = {}
    for store in (1, 0):
        ctx.set_option(logfx.OPT_STORE_Z, store)
        try:
            outs, reps = ctx.extract_batch(devs, params, bits=11, report=True)
        finally:
            ctx.set_option(logfx.OPT_STORE_Z, 1)
        torch.cuda.synchronize()
        res[store] = ([o.cpu().numpy() for o in outs], reps)
    for a, b in zip(res[0][0], res[1][0]):
        assert np.array_equal(a, b)
    assert res[0][1] == res[1][1]
    for d, o, r in zip(devs, res[1][0], res[1][1]):
        single = ctx.extract(d, logfx.Params(*lib_t, smooth=bool(r["smoothed"]), median_size=median_size),
                             bits=11).cpu().numpy()
        assert np.array_equal(o, single)


def test_gate_decides_the_median_cascade(ctx):
    """With further median levels the gate's choice covers all of them: a
    smoothed image gets every level, an unsmoothed one none (its map passes
    the levels unchanged)."""
    import torch
    tiles = _gate_tiles()[:3]
    _, lib_t = masks()
    devs = [to_device(t) for t in tiles]
    cas = (3, 5)
    always = ctx.extract_batch(devs, logfx.Params(*lib_t, smooth=True, median_cascade=cas), bits=11)
    never = ctx.extract_batch(devs, logfx.Params(*lib_t, smooth=False), bits=11)
    gparams = logfx.Params(*lib_t, smooth=logfx.SMOOTH_GATE, median_cascade=cas)
    theta = og.init(102)
    for bias, ref in ((50.0, always), (-50.0, never)):
        theta[og.NPARAM - 1] = bias
        ctx.gate_set_params(theta)
        outs = ctx.extract_batch(devs, gparams, bits=11)
        torch.cuda.synchronize()
        for o, e in zip(outs, ref):
            assert torch.equal(o, e)


def _region_scene(gy, gx, R, seed0):
    """gy x gx gate tiles of side R, each with its own noise, side by side
    in one image (the regions' seams are part of the scene)."""
    rows = []
    for y in range(gy):
        rows.append(np.concatenate([scenes.gate_tile(seed0 + y * gx + x, size=R, twin=False)[0]
                                    for x in range(gx)], axis=1))
    return np.ascontiguousarray(np.concatenate(rows, axis=0))


def _check_regions(ctx, img, R, bits, median_size, theta_seed, path):
    """Features, logits, decisions and output of a gate_region call against
    the oracle chain (features bit for bit, logits within LOGIT_TOL, output F
    or E per region under the band rule)."""
    import torch
    from parity import compare
    gy, gx = img.shape[0] // R, img.shape[1] // R
    orc_t, lib_t = masks()
    o = run_oracle(img, orc_t, smooth=True, median_size=median_size)
    regions = [(y, x) for y in range(gy) for x in range(gx)]
    crop = lambda a, y, x: a[y * R:(y + 1) * R, x * R:(x + 1) * R]
    feats_ref = np.stack([og.features(crop(img, y, x), crop(o["Z1"], y, x), crop(o["Z2"], y, x), bits)
                          for y, x in regions])
    theta = og.init(theta_seed)
    theta[og.NPARAM - 1] = 0.0
    z0, _ = og.forward(theta, feats_ref)
    # the output bias splits the regions between both choices, well away from 0
    zs = np.sort(z0)
    k = len(zs) // 2
    theta[og.NPARAM - 1] = -float(zs[k - 1] + zs[k]) / 2 if len(zs) > 1 else 1.0
    z_ref, _ = og.forward(theta, feats_ref)
    ctx.gate_set_params(theta)
    params = logfx.Params(*lib_t, smooth=logfx.SMOOTH_GATE, median_size=median_size, gate_region=R)
    dev = to_device(img)
    feats = ctx.gate_features(dev, params, bits=bits)
    logits, dec = ctx.gate(dev, params, bits=bits)
    out, rep = ctx.extract(dev, params, bits=bits, report=True)
    torch.cuda.synchronize()
    got = feats.float().cpu().numpy().astype(np.float64)
    assert got.shape == (len(regions), 3, 128, 128)
    assert np.array_equal(got, og.bf16(feats_ref))
    logits = logits.cpu().numpy()
    dec = dec.cpu().numpy()
    assert np.all(np.abs(logits - z_ref) <= LOGIT_TOL * (1 + np.abs(z_ref))), (logits, z_ref)
    sure = np.abs(z_ref) > LOGIT_TOL
    assert np.array_equal(dec[sure], (z_ref[sure] > 0).astype(np.uint8))
    if len(regions) > 1:
        assert 0 < dec.sum() < len(regions)
    assert rep["gated"] == 1 and rep["gate_fallback"] == 0 and rep["path"] == path
    assert rep["regions"] == len(regions) and rep["regions_smoothed"] == int(dec.sum())
    assert rep["sigma_g"] == pytest.approx(list(o["stats"][:2]), rel=1e-12)
    ref = o["E"].copy()
    for q, (y, x) in enumerate(regions):
        if dec[q]:
            ref[y * R:(y + 1) * R, x * R:(x + 1) * R] = crop(o["F"], y, x)
    compare(out.cpu().numpy(), {**o, "F": ref}, smooth=True, median_size=median_size)


# 144: region rows start inside a pass-2 column word (bit 16) and region
# columns inside tiles, so both the per-pixel choice across a word's region
# boundary and tiles spanning regions are exercised
@pytest.mark.parametrize("gy,gx,R,median_size", [(2, 4, 256, 5), (4, 2, 128, 3), (1, 1, 384, 5), (2, 4, 144, 5),
                                                 (4, 2, 144, 3)])
def test_gate_regions_seamless(ctx, gy, gx, R, median_size):
    """gate_region: one image, one global deviation per mask, and a gate
    decision per R x R region.  The features of each region are the oracle's
    features of that region's part of the whole image's crossing maps (bit
    for bit); the logits match the oracle network; the output is the
    oracle's smoothed map F in the smoothed regions and its unsmoothed map E
    elsewhere (band rule), with the median reading across region borders."""
    img = _region_scene(gy, gx, R, 20_000 + 97 * R)
    _check_regions(ctx, img, R, 11, median_size, 103, logfx.PATH_INT32)


def test_gate_regions_fp64_path(ctx):
    """The same on the FP64 path: 16-bit pixels whose LoG sums leave int32,
    2 x 4 regions of 128^2 with different noise levels."""
    rng = np.random.default_rng(404)
    base = rng.integers(20000, 40000, (256, 512)).astype(np.float64)
    for y in range(2):
        for x in range(4):
            base[y * 128:(y + 1) * 128, x * 128:(x + 1) * 128] += \
                rng.normal(0, 300.0 * (1 + 3 * ((y * 4 + x) % 3)), (128, 128))
    img = np.clip(np.rint(base), 0, 65535).astype(np.uint16)
    _check_regions(ctx, img, 128, 16, 5, 107, logfx.PATH_FP64)


def test_gate_regions_without_gate_parameters():
    """With no gate parameters a gate_region call falls back to always
    smoothing, as GATE does: the ALWAYS output, gate_fallback set, no
    regions reported."""
    import torch
    _, lib_t = masks()
    img = to_device(_region_scene(1, 2, 128, 31_000))
    with logfx.Context(0) as c:
        out, rep = c.extract(img, logfx.Params(*lib_t, smooth=logfx.SMOOTH_GATE, gate_region=128), bits=11,
                             report=True)
        ref = c.extract(img, logfx.Params(*lib_t, smooth=True), bits=11)
        torch.cuda.synchronize()
    assert rep["gate_fallback"] == 1 and rep["gated"] == 0 and rep["regions"] == 0 and rep["smoothed"] == 1
    assert torch.equal(out, ref)


def test_gate_regions_refused_in_batches(ctx):
    """gate_region belongs to single-image calls."""
    _, lib_t = masks()
    ctx.gate_set_params(og.init(5))
    img = to_device(np.zeros((256, 256), np.uint16))
    params = logfx.Params(*lib_t, smooth=logfx.SMOOTH_GATE, gate_region=128)
    with pytest.raises(logfx.LogfxError) as e:
        ctx.extract_batch([img, img], params, bits=11)
    assert e.value.code == logfx.EINVAL


def test_gate_regions_full_width_band(ctx):
    """The seamless mode at the four-band workload's shape: a 4096 x 16384
    strip of a band (16384 columns, 2048^2 regions, 2 x 8 of them) with its
    own noise per region, the committed gate parameters, and the launch
    configuration the benchmark times.  Decisions follow the oracle network
    on the oracle's region features (outside |logit| < tolerance); the output
    is F or E per region under the band rule."""
    import torch
    from parity import compare
    R = 2048
    img = scenes.regional_noise_scene(4096, 16384, R, seed=6)
    orc_t, lib_t = masks()
    o = run_oracle(img, orc_t, smooth=True)
    gy, gx = img.shape[0] // R, img.shape[1] // R
    regions = [(y, x) for y in range(gy) for x in range(gx)]
    crop = lambda a, y, x: a[y * R:(y + 1) * R, x * R:(x + 1) * R]
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    ctx.gate_load(os.path.join(root, "paper_1304_3992_amd", "gate_weights.bin"))
    theta = ctx.gate_get_params().astype(np.float64)
    feats_ref = np.stack([og.features(crop(img, y, x), crop(o["Z1"], y, x), crop(o["Z2"], y, x), 11)
                          for y, x in regions])
    z_ref, _ = og.forward(theta, feats_ref)
    params = logfx.Params(*lib_t, smooth=logfx.SMOOTH_GATE, gate_region=R)
    dev = to_device(img)
    out, rep = ctx.extract(dev, params, bits=11, report=True)
    logits, dec = ctx.gate(dev, params, bits=11)
    torch.cuda.synchronize()
    logits, dec = logits.cpu().numpy(), dec.cpu().numpy()
    assert np.all(np.abs(logits - z_ref) <= LOGIT_TOL * (1 + np.abs(z_ref))), (logits, z_ref)
    sure = np.abs(z_ref) > LOGIT_TOL
    assert np.array_equal(dec[sure], (z_ref[sure] > 0).astype(np.uint8))
    assert rep["regions"] == len(regions) and rep["regions_smoothed"] == int(dec.sum())
    ref = o["E"].copy()
    for q, (y, x) in enumerate(regions):
        if dec[q]:
            ref[y * R:(y + 1) * R, x * R:(x + 1) * R] = crop(o["F"], y, x)
    info = compare(out.cpu().numpy(), {**o, "F": ref}, smooth=True)
    print("full-width band:", int(dec.sum()), "of", len(regions), "regions smoothed;", info)
