"""Pins of the FP64 surrogate-network oracle.

Each check compares the oracle with something other than its own formulas:
tabulated values of the standard normal distribution, scipy's normal CDF,
central finite differences, an affine special case evaluated by plain matrix
products, and properties of Adam stated by Kingma & Ba (2015).
"""
import math

import numpy as np
import pytest
from scipy.stats import norm

from oracle import mlp_oracle as M

TINY = (3, 5, 4, 6, 2)


def test_param_count_of_the_surrogate_architecture():
    # 19*256+256 + 2*(256*256+256) + 256*64+64
    assert M.param_count() == 153152


def test_gelu_tabulated_values():
    # gelu(z) = z Phi(z); Phi(1) = 0.8413447460685429, Phi(2) = 0.9772498680518208 (normal table)
    assert abs(M.gelu(1.0) - 0.8413447460685429) < 1e-15
    assert abs(M.gelu(-1.0) + (1.0 - 0.8413447460685429)) < 1e-15
    assert abs(M.gelu(2.0) - 2 * 0.9772498680518208) < 1e-15
    assert M.gelu(0.0) == 0.0
    z = np.linspace(-6, 6, 97)
    assert np.abs(M.gelu(z) - z * norm.cdf(z)).max() < 1e-14


def test_gelu_grad_by_central_differences():
    z = np.linspace(-5, 5, 41)
    h = 1e-5
    fd = (M.gelu(z + h) - M.gelu(z - h)) / (2 * h)
    assert np.abs(M.gelu_grad(z) - fd).max() < 1e-9
    assert abs(M.gelu_grad(0.0) - 0.5) < 1e-15


def _tiny(seed=0, n=7):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.7, M.param_count(TINY))
    X = rng.normal(0, 1, (n, TINY[0]))
    Y = rng.normal(0, 1, (n, TINY[-1]))
    return p, X, Y


def test_loss_gradient_matches_central_differences():
    p, X, Y = _tiny()
    loss, g = M.loss_grad(p, X, Y, TINY)
    h = 1e-6
    fd = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        fd[i] = (M.loss_grad(p + e, X, Y, TINY)[0] - M.loss_grad(p - e, X, Y, TINY)[0]) / (2 * h)
    assert np.abs(g - fd).max() <= 1e-6 * np.abs(fd).max()
    assert loss > 0


def test_affine_regime_equals_plain_matrix_chain():
    """With every hidden pre-activation above 12, gelu(z) = z to double precision,
    so the network is the affine map W4 (W3 (W2 (W1 x + b1) + b2) + b3) + b4."""
    rng = np.random.default_rng(3)
    Ws = [rng.uniform(0.0, 0.1, (TINY[i + 1], TINY[i])) for i in range(4)]
    bs = [np.full(TINY[i + 1], 15.0) if i < 3 else rng.normal(0, 1, TINY[-1]) for i in range(4)]
    p = np.concatenate([np.concatenate([W.ravel(), b]) for W, b in zip(Ws, bs)])
    X = rng.uniform(0, 1, (5, TINY[0]))
    y = M.forward(p, X, TINY)
    ref = X.T
    for W, b in zip(Ws, bs):
        ref = W @ ref + b[:, None]
    assert np.abs(y - ref.T).max() < 1e-12


def test_loss_is_zero_at_the_targets():
    p, X, _ = _tiny(1)
    Y = M.forward(p, X, TINY)
    loss, g = M.loss_grad(p, X, Y, TINY)
    assert loss == 0.0 and not g.any()


def test_adam_first_step_is_lr_times_sign():
    """Bias correction makes the first step lr g / (|g| + eps) (Kingma & Ba, Sec. 2.1:
    the effective step is bounded by the step size)."""
    g = np.array([3.0, -0.2, 1e-3, -50.0])
    p, m, v = M.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    assert np.allclose(p, -0.01 * np.sign(g), rtol=1e-5, atol=0)


def test_adam_is_invariant_to_gradient_scale():
    rng = np.random.default_rng(5)
    gs = rng.normal(0, 1, (6, 10))
    pa = pb = np.zeros(10)
    ma = va = mb = vb = np.zeros(10)
    for t, g in enumerate(gs, start=1):
        pa, ma, va = M.adam_step(pa, g, ma, va, t, lr=0.05, eps=0.0)
        pb, mb, vb = M.adam_step(pb, 1000.0 * g, mb, vb, t, lr=0.05, eps=0.0)
    assert np.abs(pa - pb).max() < 1e-13


@pytest.mark.parametrize("target", [3.0, -1.5])
def test_adam_minimises_a_quadratic(target):
    p, m, v = np.zeros(1), np.zeros(1), np.zeros(1)
    for t in range(1, 3001):
        p, m, v = M.adam_step(p, p - target, m, v, t, lr=0.02)
    assert abs(p[0] - target) < 1e-3
