"""FP64 reference of the tuner's cost model (TEST INFRASTRUCTURE ONLY).

A multilayer perceptron in -> H -> H -> 1 with ReLU hidden layers, the
mean-squared-error loss and one Adam update (Kingma & Ba, "Adam: a method
for stochastic optimization", 2015), written as plain numpy matrix algebra.
Parameters are packed like the HIP implementation's: W1[in][H], b1[H],
W2[H][H], b2[H], w3[H], b3.  The backward pass is the chain rule written out
layer by layer; tests pin it against central finite differences.
"""
from __future__ import annotations

import numpy as np


def n_params(in_dim: int, hidden: int) -> int:
    return in_dim * hidden + hidden + hidden * hidden + hidden + hidden + 1


def unpack(p: np.ndarray, in_dim: int, hidden: int):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + in_dim * hidden].reshape(in_dim, hidden); o += in_dim * hidden
    b1 = p[o:o + hidden]; o += hidden
    W2 = p[o:o + hidden * hidden].reshape(hidden, hidden); o += hidden * hidden
    b2 = p[o:o + hidden]; o += hidden
    w3 = p[o:o + hidden]; o += hidden
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def forward(X, p, in_dim: int, hidden: int):
    W1, b1, W2, b2, w3, b3 = unpack(p, in_dim, hidden)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1 + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2 + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w3 + b3
    return y, (X, z1, h1, z2, h2)


def loss_grad(X, T, p, in_dim: int, hidden: int):
    """(loss, gradient) of mean_b (y_b - t_b)^2."""
    W1, b1, W2, b2, w3, b3 = unpack(p, in_dim, hidden)
    y, (X, z1, h1, z2, h2) = forward(X, p, in_dim, hidden)
    T = np.asarray(T, dtype=np.float64)
    B = X.shape[0]
    e = y - T
    loss = float(np.mean(e * e))
    dy = 2.0 * e / B
    g_w3 = h2.T @ dy
    g_b3 = np.sum(dy)
    dh2 = np.outer(dy, w3) * (z2 > 0)
    g_W2 = h1.T @ dh2
    g_b2 = dh2.sum(axis=0)
    dh1 = (dh2 @ W2.T) * (z1 > 0)
    g_W1 = X.T @ dh1
    g_b1 = dh1.sum(axis=0)
    g = np.concatenate([g_W1.ravel(), g_b1, g_W2.ravel(), g_b2, g_w3, [g_b3]])
    return loss, g


def adam(p, g, m, v, lr, beta1, beta2, eps, step):
    """One Adam update; returns (p, m, v)."""
    m = beta1 * np.asarray(m, dtype=np.float64) + (1 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return np.asarray(p, dtype=np.float64) - lr * mh / (np.sqrt(vh) + eps), m, v
