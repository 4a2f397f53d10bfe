"""Pins of the proposer oracle: bfloat16 rounding against torch's conversion, gradients
against central finite differences (FP64 function), the loss in closed form, and the
features on fields with known values."""
import math

import numpy as np
import pytest

P, H, N = 24, 4, 16


def _params(orc, rng, scale=0.2):
    return rng.normal(scale=scale, size=orc.mlp_nparams())


def test_bf16_round_matches_torch(orc):
    import torch
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=2000), rng.normal(size=200) * 1e-30, rng.normal(size=200) * 1e30,
                        [0.0, -0.0, 1.0, -1.0, 1.00390625, 1.01171875]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    got = np.array([orc.bf16_round(float(v)) for v in x])
    assert np.array_equal(got, ref)


def test_gradient_finite_differences(orc):
    rng = np.random.default_rng(1)
    params = _params(orc, rng)
    X = rng.normal(size=(6, 192))
    y = np.array([0, 1, 2, 1, 1, 0])
    w = (2.0, 1.0, 3.0)
    _, g = orc.mlp_loss_grad(params, X, y, w, bf16=False)
    idx = rng.choice(len(params), size=150, replace=False)
    for i in idx:
        h = 1e-6
        pp, pm = params.copy(), params.copy()
        pp[i] += h
        pm[i] -= h
        lp, _ = orc.mlp_loss_grad(pp, X, y, w, bf16=False)
        lm, _ = orc.mlp_loss_grad(pm, X, y, w, bf16=False)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-8, (i, fd, g[i])


def test_loss_closed_form(orc):
    # zero weights: logits = b3 for every sample; weighted mean cross-entropy of softmax(b3)
    params = np.zeros(orc.mlp_nparams())
    b3 = np.array([0.3, -1.2, 0.7])
    params[-3:] = b3
    X = np.random.default_rng(2).normal(size=(5, 192))
    y = np.array([0, 2, 2, 1, 0])
    w = np.array([1.0, 0.5, 2.0])
    loss, g = orc.mlp_loss_grad(params, X, y, w, bf16=False)
    lse = math.log(np.exp(b3).sum())
    ref = sum(w[t] * (lse - b3[t]) for t in y) / sum(w[t] for t in y)
    assert abs(loss - ref) < 1e-14
    assert np.allclose(orc.mlp_forward(params, X, bf16=False), np.tile(b3, (5, 1)))


def test_features_closed_form(orc):
    gamma, B = 1.4, 0.0
    # uniform state: mean rho, zero gradient, mean p
    u = np.zeros((5, P, P, P))
    rho, p = 1.3, 0.8
    u[0] = rho
    u[4] = p / (gamma - 1)
    f = orc.features(u, gamma, B, 1.0, 2.0, 1e-3)
    assert np.allclose(f[0::3], rho - 1.0) and np.allclose(f[1::3], 0.0) and np.allclose(f[2::3], p / 2.0 - 1.0)
    # density linear in x (slope a per cell): central and one-sided differences are exact
    a = 2e-3
    x = np.arange(P) - H
    u[0] = 1.0 + a * x[None, None, :]
    f = orc.features(u, gamma, B, 1.0, 2.0, 1e-3)
    assert np.allclose(f[1::3], math.log(1.0 + a / 1e-3), rtol=1e-13)
    # sub-cube means of rho follow the sub-cube centre
    sx = np.arange(64) % 4
    assert np.allclose(f[0::3], a * (4 * sx + 1.5))
