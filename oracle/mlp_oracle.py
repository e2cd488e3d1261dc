"""Plain FP64 CPU reference of the learned outer-step controller's network.

TEST INFRASTRUCTURE ONLY.  Only the test-suite may import or run this
file; the product path never calls it.

The controller maps 16 features of an outer step to 3 outputs (log of the
next inner tolerance, log of the next inner iteration budget, log of the
next primal weight) with a fully connected network 16 -> 64 -> 64 -> 3,
ReLU after the two hidden layers, trained by mean-squared error with Adam.
Parameters are one flat vector in the order W1 (16x64, row-major: input
index major), b1 (64), W2 (64x64), b2 (64), W3 (64x3), b3 (3).
"""

from __future__ import annotations

import numpy as np

N_IN, N_H, N_OUT = 16, 64, 3
SHAPES = [(N_IN, N_H), (N_H,), (N_H, N_H), (N_H,), (N_H, N_OUT), (N_OUT,)]
N_PARAMS = sum(int(np.prod(s)) for s in SHAPES)  # 5443


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, k = [], 0
    for s in SHAPES:
        size = int(np.prod(s))
        out.append(theta[k:k + size].reshape(s))
        k += size
    return out


def forward(theta, X):
    """Returns the outputs (B x 3) and the hidden pre-activations."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1 + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2 + b2
    h2 = np.maximum(z2, 0.0)
    return h2 @ W3 + b3, (X, z1, h1, z2, h2)


def loss(theta, X, Y):
    """Mean over samples and outputs of the squared error."""
    out, _ = forward(theta, X)
    d = out - np.asarray(Y, dtype=np.float64)
    return float(np.mean(d * d))


def gradient(theta, X, Y):
    """Gradient of ``loss`` by the chain rule, written out layer by layer."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    out, (X, z1, h1, z2, h2) = forward(theta, X)
    B = X.shape[0]
    g_out = 2.0 * (out - np.asarray(Y, dtype=np.float64)) / (B * N_OUT)
    gW3 = h2.T @ g_out
    gb3 = g_out.sum(axis=0)
    g_h2 = g_out @ W3.T
    g_z2 = g_h2 * (z2 > 0.0)
    gW2 = h1.T @ g_z2
    gb2 = g_z2.sum(axis=0)
    g_h1 = g_z2 @ W2.T
    g_z1 = g_h1 * (z1 > 0.0)
    gW1 = X.T @ g_z1
    gb1 = g_z1.sum(axis=0)
    return np.concatenate([g.ravel() for g in (gW1, gb1, gW2, gb2, gW3, gb3)])


def adam_step(theta, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba); t counts from 1.  Returns the new
    (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
