"""Pins for the oracle of the learned depth prefilter.

* a convolution equals scipy's 2-d correlation summed over input channels
  (stride 2 = the stride-1 result at even positions);
* im2col/col2im and up2/its backward are adjoint pairs;
* every parameter gradient of the loss matches central finite differences
  in float64;
* a zero head leaves valid depth unchanged and invalid depth at 0;
* one Adam step on a quadratic has a closed form;
* bfloat16 rounding is round-to-nearest-even (hand values, torch's cast).
"""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import denoise as D


def _rand_params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    P = D.init_params(seed)
    for k in P:
        if k.endswith(".b") or k.startswith("head"):
            P[k] = rng.standard_normal(P[k].shape) * 0.1 * scale
    return P


@pytest.mark.parametrize("stride", [1, 2])
def test_conv_is_channel_summed_correlation(stride):
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 12, 10, 3))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    y = D.conv(x, w, b, stride)
    for n in range(2):
        for co in range(4):
            ref = sum(correlate2d(x[n, :, :, ci], w[co, :, :, ci], mode="same") for ci in range(3)) + b[co]
            assert np.allclose(y[n, :, :, co], ref[::stride, ::stride], atol=1e-12)


def test_adjoint_pairs():
    rng = np.random.default_rng(2)
    for stride in (1, 2):
        x = rng.standard_normal((2, 9, 8, 3))
        c = rng.standard_normal(D.im2col(x, stride).shape)
        assert np.isclose(np.sum(D.im2col(x, stride) * c), np.sum(x * D.col2im(c, x.shape, stride)))
    x = rng.standard_normal((1, 4, 6, 2))
    y = rng.standard_normal((1, 8, 12, 2))
    assert np.isclose(np.sum(D.up2(x) * y), np.sum(x * D.up2_backward(y)))


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(3)
    P = _rand_params(3)
    depth = rng.uniform(0.5, 3.5, (2, 16, 16))
    depth[0, 3:5, 7:9] = 0.0                         # invalid input pixels
    target = depth + rng.normal(0, 0.05, depth.shape)
    target[1, 10, 2:6] = 0.0                         # invalid target pixels
    out, c = D.forward(P, depth)
    loss, g, n = D.loss_and_grad_out(out, depth, target)
    assert n == int(((depth > 0) & (target > 0)).sum())
    G = D.backward(P, c, g)
    assert set(G) == set(P)
    h = 1e-6
    worst = 0.0
    for k in P:
        flat = P[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = D.loss_fn(P, depth, target)
            flat[idx] = old - h
            lm = D.loss_fn(P, depth, target)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = G[k].reshape(-1)[idx]
            err = abs(fd - an) / max(abs(fd), abs(an), 1e-3)
            worst = max(worst, err)
            assert err < 1e-5, (k, idx, fd, an)
    assert worst < 1e-5


def test_zero_head_is_identity():
    rng = np.random.default_rng(4)
    P = D.init_params(4)
    depth = rng.uniform(0.3, 4.0, (1, 24, 32))
    depth[0, :3] = 0.0
    out, _ = D.forward(P, depth)
    assert np.array_equal(out, np.where(depth > 0, depth, 0.0))
    # and so the loss gradient reaches only the head's parameters
    target = depth + 0.01
    _, g, _ = D.loss_and_grad_out(out, depth, target)
    _, c = D.forward(P, depth)
    G = D.backward(P, c, g)
    assert all(np.all(G[k] == 0) for k in G if not k.startswith("head"))
    assert np.any(G["head.w"] != 0)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(5)
    p0 = rng.standard_normal(50)
    ctr = rng.standard_normal(50)
    P = {"p": p0.copy()}
    state = {}
    D.adam_step(P, {"p": p0 - ctr}, state, 1)
    g = p0 - ctr
    # m_hat = g, v_hat = g^2 after the first step
    want = p0 - D.ADAM["lr"] * g / (np.abs(g) + D.ADAM["eps"])
    assert np.allclose(P["p"], want, rtol=0, atol=1e-15)
    # second step with the same gradient: m_hat = g, v_hat = g^2 again
    D.adam_step(P, {"p": p0 - ctr}, state, 2)
    assert np.allclose(P["p"], want - D.ADAM["lr"] * g / (np.abs(g) + D.ADAM["eps"]), atol=1e-15)


def test_bf16_rounding():
    one = 1.0
    vals = np.array([one, one + 2.0 ** -8, one + 3 * 2.0 ** -8, one + 2.0 ** -8 + 2.0 ** -20, -2.5, 0.0], np.float32)
    want = np.array([one, one, one + 2.0 ** -6, one + 2.0 ** -7, -2.5, 0.0], np.float32)
    assert np.array_equal(D.to_bf16(vals), want)
    import torch
    x = np.random.default_rng(6).standard_normal(10000).astype(np.float32) * 100
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(D.to_bf16(x), ref)


def test_parameter_count():
    # 896 + 18496 + 36928 + 73856 + 73792 + 36928 + 18464 + 289
    assert D.n_params(D.init_params()) == 259649


def test_input_channels():
    d = np.array([[[1.0, 1.0, 0.0, 2.0],
                   [1.0, 1.3, 1.0, 2.0],
                   [0.0, 1.0, 1.0, 2.0]]])
    x = D.make_input(d)
    assert np.array_equal(x[..., 0], d / 4) and np.array_equal(x[..., 1], (d > 0) * 1.0)
    # pixel (1, 1): valid 3x3 neighbours 1, 1, 1, 1.3, 1, 1, 1 (two holes) -> mean 7.3 / 7
    assert np.isclose(x[0, 1, 1, 2], (1.3 - 7.3 / 7) / 0.05)
    # corner (0, 0): neighbours 1, 1, 1, 1.3 -> mean 4.3 / 4; a hole stays 0
    assert np.isclose(x[0, 0, 0, 2], (1.0 - 4.3 / 4) / 0.05) and x[0, 0, 2, 2] == 0
    # a constant valid patch has zero deviation
    assert np.allclose(D.make_input(np.full((1, 5, 5), 2.5))[..., 2], 0)


def test_activation_shapes_and_skips():
    P = D.init_params(7)
    _, c = D.forward(P, np.ones((1, 32, 48)))
    shapes = {k: c[k].shape[1:] for k in ("e1", "e2", "e3", "e4", "d3", "d2", "d1")}
    assert shapes == {"e1": (32, 48, 32), "e2": (16, 24, 64), "e3": (8, 12, 64), "e4": (4, 6, 128),
                      "d3": (8, 12, 64), "d2": (16, 24, 64), "d1": (32, 48, 32)}
    # a decoder level with zero conv weights and bias passes its skip through the relu
    P["d1.w"][:] = 0.0
    _, c = D.forward(P, np.ones((1, 32, 48)))
    assert np.array_equal(c["d1"], c["e1"])
