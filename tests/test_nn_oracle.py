"""Pins of the FP64 NumPy reference of the learned scorer (CPU only)."""
import numpy as np
import pytest
import torch

from oracle import nn_ref as nn


def _batch(B, seed=0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((B, 21, 21)), rng.standard_normal((B, 16)), (rng.random(B) < 0.5).astype(float)


def test_param_count_and_layout():
    assert nn.n_params() == 144 + 16 + 4608 + 32 + 9216 + 32 + 73728 + 64 + 1024 + 64 + 8192 + 64 + 64 + 1
    th = nn.init_params(1)
    np.testing.assert_array_equal(nn.flatten(nn.unflatten(th)), th)


def test_im2col_adjoint_and_direct_convolution():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 7, 8, 3))
    for stride in (1, 2):
        c = nn.im2col(x, stride)
        y = rng.standard_normal(c.shape)
        assert np.isclose((c * y).sum(), (x * nn.col2im(y, x.shape, stride)).sum(), rtol=1e-12)
        w = rng.standard_normal((27, 4))
        out = c @ w
        # direct zero-padded cross-correlation with the same weight layout
        W4 = w.reshape(3, 3, 3, 4)
        Ho, Wo = out.shape[1], out.shape[2]
        ref = np.zeros_like(out)
        for b in range(2):
            for oy in range(Ho):
                for ox in range(Wo):
                    for ky in range(3):
                        for kx in range(3):
                            iy, ix = oy * stride + ky - 1, ox * stride + kx - 1
                            if 0 <= iy < 7 and 0 <= ix < 8:
                                ref[b, oy, ox] += x[b, iy, ix] @ W4[ky, kx]
        np.testing.assert_allclose(out, ref, atol=1e-12)


def test_bce_and_logit_gradient_closed_form():
    z = np.array([-3.0, -0.2, 0.0, 0.7, 4.0])
    y = np.array([0.0, 1.0, 1.0, 0.0, 1.0])
    s = 1 / (1 + np.exp(-z))
    assert nn.bce_with_logits(z, y) == pytest.approx(np.mean(-(y * np.log(s) + (1 - y) * np.log(1 - s))), rel=1e-14)
    # big logits stay finite
    assert np.isfinite(nn.bce_with_logits(np.array([800.0, -800.0]), np.array([0.0, 1.0])))
    # for a net whose last layers are linear, dL/db7 = mean(sigmoid(z) - y)
    th = nn.init_params(2)
    X, F, Y = _batch(6, 1)
    loss, g = nn.loss_and_grad(th, X, F, Y)
    z = nn.forward(th, X, F)
    assert g[-1] == pytest.approx(np.mean(1 / (1 + np.exp(-z)) - Y), rel=1e-12)


def test_gradients_match_central_differences():
    th = nn.init_params(5) * 0.5
    p = nn.unflatten(th)
    for k in p:
        if k.startswith("b"):
            p[k] = np.random.default_rng(9).standard_normal(p[k].shape) * 0.1   # non-zero biases
    th = nn.flatten(p)
    X, F, Y = _batch(3, 2)
    loss, g = nn.loss_and_grad(th, X, F, Y)
    rng = np.random.default_rng(4)
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in nn.LAYERS])
    idx = np.concatenate([rng.choice(np.arange(offs[i], offs[i + 1]), min(12, offs[i + 1] - offs[i]), replace=False)
                          for i in range(len(nn.LAYERS))])
    h = 1e-6
    for i in idx:
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd = (nn.bce_with_logits(nn.forward(tp, X, F), Y) - nn.bce_with_logits(nn.forward(tm, X, F), Y)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_adam_first_step_is_signed_lr():
    th = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -1e-3, 4.0])
    t1, m, v = nn.adam_step(th, np.zeros(3), np.zeros(3), g, 1, 1e-2)
    np.testing.assert_allclose(t1, th - 1e-2 * np.sign(g), rtol=0, atol=1e-7)


def test_bf16_round_matches_torch():
    x = np.random.default_rng(0).standard_normal(10000) * np.exp(np.random.default_rng(1).uniform(-20, 20, 10000))
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(nn.bf16_round(x), ref)
