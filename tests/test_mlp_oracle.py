"""Pins of the controller network's CPU reference (oracle/mlp_oracle.py):
central finite differences of the loss, the linear regime in closed form,
and Adam's first step."""

import numpy as np

from oracle import mlp_oracle as M


def _theta(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.normal(scale=scale, size=M.N_PARAMS)


def test_parameter_count():
    assert M.N_PARAMS == 16 * 64 + 64 + 64 * 64 + 64 + 64 * 3 + 3 == 5443


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    th = _theta(2)
    X = rng.normal(size=(9, 16))
    Y = rng.normal(size=(9, 3))
    g = M.gradient(th, X, Y)
    idx = rng.choice(M.N_PARAMS, size=60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(th)
        e[i] = h
        fd = (M.loss(th + e, X, Y) - M.loss(th - e, X, Y)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), i


def test_linear_regime_closed_form():
    """With every hidden pre-activation positive the network is affine:
    out = ((X W1 + b1) W2 + b2) W3 + b3."""
    th = np.abs(_theta(3, 0.1))
    W1, b1, W2, b2, W3, b3 = M.unpack(th)
    X = np.abs(np.random.default_rng(4).normal(size=(5, 16)))
    out, _ = M.forward(th, X)
    np.testing.assert_allclose(out, ((X @ W1 + b1) @ W2 + b2) @ W3 + b3, rtol=1e-12)


def test_relu_gate_blocks_gradient():
    """A hidden unit that is off for every sample gets no gradient."""
    th = _theta(5)
    W1, b1, W2, b2, W3, b3 = M.unpack(th)
    b1[7] = -1e6           # unit 7 of the first layer is always off
    g = M.gradient(th, np.random.default_rng(6).normal(size=(4, 16)), np.zeros((4, 3)))
    gW1 = g[:16 * 64].reshape(16, 64)
    assert np.all(gW1[:, 7] == 0.0) and g[16 * 64 + 7] == 0.0


def test_adam_first_step_is_signed_lr():
    """At t = 1 the bias-corrected moments give a step of lr * g / (|g| + eps)."""
    th = np.zeros(4)
    g = np.array([1e-3, -2.0, 0.5, 0.0])
    th1, m, v = M.adam_step(th, g, np.zeros(4), np.zeros(4), 1, 0.01)
    np.testing.assert_allclose(th1, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
