"""Pins of the gate oracle (no GPU): rounding, convolution, gradients and the
optimiser step against library routines and finite differences; features
against a per-cell brute force.  The labelling rule has its own pins in
test_gate_labels.py."""
import numpy as np
import pytest
import torch

from oracle import gate


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(0, 1, 5000), rng.normal(0, 1e-3, 5000), [0.0, -0.0, 1.0, 3.0],
                        np.float32([1.00390625, 1.01171875, -2.0078125])])  # exact ties
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(gate.bf16(x.astype(np.float32)), ref)


def test_conv_matches_torch_and_backward_matches_autograd():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(2, 3, 16, 16))
    w = rng.normal(size=(5, 3, 3, 3))
    b = rng.normal(size=5)
    xt = torch.tensor(x, requires_grad=True)
    wt = torch.tensor(w, requires_grad=True)
    bt = torch.tensor(b, requires_grad=True)
    yt = torch.nn.functional.conv2d(xt, wt, bt, stride=2, padding=1)
    y = gate.conv_s2(x, w, b)
    assert np.allclose(y, yt.detach().numpy(), rtol=1e-12, atol=1e-12)
    g = rng.normal(size=y.shape)
    yt.backward(torch.tensor(g))
    dx, dw, db = gate.conv_s2_backward(x, w, g)
    assert np.allclose(dx, xt.grad.numpy(), rtol=1e-12, atol=1e-12)
    assert np.allclose(dw, wt.grad.numpy(), rtol=1e-12, atol=1e-12)
    assert np.allclose(db, bt.grad.numpy(), rtol=1e-12, atol=1e-12)


def test_gradient_matches_central_differences():
    """FP64 path (no rounding): the analytic gradient of the mean BCE equals
    central finite differences on parameters of every layer."""
    rng = np.random.default_rng(3)
    theta = gate.init(7) * 0.5
    theta[-1] = 0.1
    feats = rng.random((3, 3, 128, 128))
    y = np.array([1.0, 0.0, 1.0])
    loss, g = gate.backward(theta, feats, y, bf=False)
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in gate.SHAPES])
    idx = [offs[k] + j for k in range(len(gate.SHAPES)) for j in (0, 3)
           if offs[k] + j < offs[k + 1]]
    for i in idx:
        h = 1e-6 * max(1.0, abs(theta[i]))
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (gate.bce(gate.forward(tp, feats, False)[0], y) -
              gate.bce(gate.forward(tm, feats, False)[0], y)) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-5, abs=1e-9), i


def test_zero_weights_give_the_bias():
    theta = np.zeros(gate.NPARAM)
    theta[-1] = 0.37
    feats = np.random.default_rng(4).random((2, 3, 128, 128))
    z, _ = gate.forward(theta, feats)
    assert np.array_equal(z, [0.37, 0.37])


def test_adamw_matches_torch():
    rng = np.random.default_rng(5)
    theta = rng.normal(size=50)
    grads = [rng.normal(size=50) for _ in range(3)]
    p = torch.tensor(theta.copy(), requires_grad=True)
    opt = torch.optim.AdamW([p], lr=1e-2, betas=(0.9, 0.999), eps=1e-8, weight_decay=1e-4)
    m = np.zeros(50)
    v = np.zeros(50)
    for step, g in enumerate(grads, 1):
        p.grad = torch.tensor(g)
        opt.step()
        theta, m, v = gate.adamw(theta, g, m, v, step, 1e-2)
    assert np.allclose(theta, p.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_features_match_per_cell_brute_force():
    rng = np.random.default_rng(6)
    for H, W in [(200, 300), (64, 130), (128, 128), (5, 7)]:
        img = rng.integers(0, 2048, (H, W))
        Z1 = (rng.random((H, W)) < 0.3) * 1.0
        Z2 = (rng.random((H, W)) < 0.6) * 2.0
        f = gate.features(img, Z1, Z2, 11)
        for cy in range(0, 128, 37):
            for cx in range(0, 128, 41):
                ys = [y for y in range(H) if y * 128 // H == cy]
                xs = [x for x in range(W) if x * 128 // W == cx]
                if not ys or not xs:
                    assert (f[:, cy, cx] == 0).all()
                    continue
                blk = np.ix_(ys, xs)
                assert f[0, cy, cx] == pytest.approx(img[blk].mean() / 2047, rel=1e-12)
                assert f[1, cy, cx] == pytest.approx((Z1[blk] != 0).mean(), rel=1e-12)
                assert f[2, cy, cx] == pytest.approx((Z2[blk] != 0).mean(), rel=1e-12)
