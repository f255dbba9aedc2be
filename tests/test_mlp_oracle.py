"""Pins of the FP64 warm-start network oracle: analytic gradients against
central finite differences, the exact-erf GELU against scipy's normal CDF,
standardisation statistics against numpy, and Adam's first step (which
moves every parameter by lr times the sign of its gradient)."""
import math

import numpy as np
import pytest

import oracle


def init_params(rng):
    n = oracle.mlp_param_count()
    assert n == 64 * 32 + 64 + 64 * 64 + 64 + 3 * 64 + 3 == 6467
    return rng.normal(scale=0.3, size=n)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    p = init_params(rng)
    x = rng.normal(size=(7, 32)) * 3 + 1
    t = rng.normal(size=(7, 3))
    mean, std = oracle.mlp_norm_stats(x)
    loss, g = oracle.mlp_loss_grad(p, mean, std, x, t)
    idx = rng.choice(p.size, 300, replace=False)
    idx = np.concatenate([idx, [0, 2047, 2048, 2111, 6211, 6272, 6463, 6466]])
    def central(k, eps):
        pp, pm = p.copy(), p.copy()
        pp[k] += eps
        pm[k] -= eps
        return (oracle.mlp_loss_grad(pp, mean, std, x, t, False)[0] -
                oracle.mlp_loss_grad(pm, mean, std, x, t, False)[0]) / (2 * eps)

    for k in idx:
        # Richardson extrapolation of central differences (error O(eps^4))
        fd = (4 * central(k, 5e-5) - central(k, 1e-4)) / 3
        assert abs(fd - g[k]) <= 1e-7 * max(abs(g[k]), 1e-3), (k, fd, g[k])


def test_forward_closed_form_pieces():
    """Zero hidden weights: every hidden unit is GELU(bias), so the output is
    b3 + W3 . GELU(b2) with GELU(z) = z Phi(z)."""
    from scipy.stats import norm
    rng = np.random.default_rng(1)
    p = np.zeros(6467)
    b1 = rng.normal(size=64)
    b2 = rng.normal(size=64)
    W3 = rng.normal(size=(3, 64))
    b3 = rng.normal(size=3)
    o = 2048
    p[o:o + 64] = b1
    o += 64 + 4096
    p[o:o + 64] = b2
    o += 64
    p[o:o + 192] = W3.reshape(-1)
    p[o + 192:] = b3
    x = rng.normal(size=(5, 32))
    y = oracle.mlp_forward(p, np.zeros(32), np.ones(32), x)
    want = b3 + W3 @ (b2 * norm.cdf(b2))
    assert np.allclose(y, want[None, :], atol=1e-12)


def test_norm_stats_match_numpy():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(1000, 32)) * np.arange(1, 33) + np.arange(32)
    mean, std = oracle.mlp_norm_stats(x)
    assert np.allclose(mean, x.mean(0), rtol=1e-13, atol=1e-12)
    assert np.allclose(std, np.sqrt(x.var(0) + 1e-12), rtol=1e-12)


def test_adam_first_step_is_signed_lr():
    rng = np.random.default_rng(3)
    p = rng.normal(size=100)
    g = rng.normal(size=100)
    m, v = np.zeros(100), np.zeros(100)
    p0 = p.copy()
    oracle.mlp_adam(p, m, v, g, 1, lr=1e-3)
    assert np.allclose(p0 - p, 1e-3 * np.sign(g) * np.abs(g) / (np.abs(g) + 1e-8), rtol=1e-12)


def test_loss_decreases_under_adam():
    rng = np.random.default_rng(4)
    p = init_params(rng) * 0.3
    x = rng.normal(size=(256, 32))
    t = np.tanh(x[:, :3]) + 0.1 * x[:, 3:6]
    mean, std = oracle.mlp_norm_stats(x)
    m, v = np.zeros_like(p), np.zeros_like(p)
    l0 = oracle.mlp_loss_grad(p, mean, std, x, t, False)[0]
    for step in range(1, 101):
        _, g = oracle.mlp_loss_grad(p, mean, std, x, t)
        oracle.mlp_adam(p, m, v, g, step, lr=3e-3)
    l1 = oracle.mlp_loss_grad(p, mean, std, x, t, False)[0]
    assert l1 < 0.3 * l0
