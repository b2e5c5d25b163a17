"""FP64 numpy oracle of the learned tuner's network -- TEST INFRASTRUCTURE.

The network (no paper passage: it is the learned-tuner extension):
    z1 = W1 x + b1, a1 = relu(z1); z2 = W2 a1 + b2, a2 = relu(z2); out = w3 . a2 + b3
loss = mean over the batch of (out - y)^2, and Adam (Kingma & Ba) with bias
correction.  Written from those definitions, independent of the HIP kernels;
pinned in the tests by finite differences of the loss, a hand-computed
network, and Adam's first-step property |update| = lr for every coordinate
with a nonzero gradient.
"""
from __future__ import annotations

import numpy as np


def unpack(params, D, H):
    p = np.asarray(params, dtype=np.float64)
    o = 0
    W1 = p[o:o + H * D].reshape(H, D); o += H * D
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    w3 = p[o:o + H]; o += H
    b3 = p[o]; o += 1
    assert o == p.size
    return W1, b1, W2, b2, w3, b3


def param_count(D, H):
    return H * D + H + H * H + H + H + 1


def forward(params, X, D, H):
    W1, b1, W2, b2, w3, b3 = unpack(params, D, H)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1.T + b1
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ W2.T + b2
    a2 = np.maximum(z2, 0.0)
    return a2 @ w3 + b3


def loss(params, X, y, D, H):
    e = forward(params, X, D, H) - np.asarray(y, dtype=np.float64)
    return float(np.mean(e * e))


def gradient(params, X, y, D, H):
    """Analytic gradient of `loss` by the chain rule, layer by layer."""
    W1, b1, W2, b2, w3, b3 = unpack(params, D, H)
    X = np.asarray(X, dtype=np.float64)
    B = X.shape[0]
    z1 = X @ W1.T + b1
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ W2.T + b2
    a2 = np.maximum(z2, 0.0)
    out = a2 @ w3 + b3
    dout = 2.0 * (out - np.asarray(y, dtype=np.float64)) / B
    g_w3 = a2.T @ dout
    g_b3 = dout.sum()
    dz2 = np.outer(dout, w3) * (z2 > 0)
    g_W2 = dz2.T @ a1
    g_b2 = dz2.sum(0)
    dz1 = (dz2 @ W2) * (z1 > 0)
    g_W1 = dz1.T @ X
    g_b1 = dz1.sum(0)
    return np.concatenate([g_W1.ravel(), g_b1, g_W2.ravel(), g_b2, g_w3, [g_b3]])


def adam_step(params, grads, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    m = beta1 * m + (1 - beta1) * grads
    v = beta2 * v + (1 - beta2) * grads * grads
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
