"""CPU oracle of the exchange selector's MLP -- TEST INFRASTRUCTURE ONLY.

A plain float64 multilayer perceptron written out with numpy, used to check
the GPU library's hand-written forward, backward and SGD kernels.  It shares
no code with them.

Network (parameters packed in this order, row-major):
    h1 = tanh(W1 x + b1)      W1: [H, D], b1: [H]
    h2 = tanh(W2 h1 + b2)     W2: [H, H], b2: [H]
    y  = W3 h2 + b3           W3: [K, H], b3: [K]
Loss over a batch of n samples: L = (1 / (2n)) * sum_i sum_k (y_ik - t_ik)^2
(the targets are per-exchange-variant log-times -- a push over the frontier
list, a push sweeping every vertex, a pull; the selector picks the variant
with the smallest prediction among those available).
SGD step: p <- p - lr * dL/dp.
"""
from __future__ import annotations

import numpy as np

D, H, K = 4, 16, 3


def n_params(d: int = D, h: int = H, k: int = K) -> int:
    return h * d + h + h * h + h + k * h + k


def unpack(p: np.ndarray, d: int = D, h: int = H, k: int = K):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + h * d].reshape(h, d); o += h * d
    b1 = p[o:o + h]; o += h
    W2 = p[o:o + h * h].reshape(h, h); o += h * h
    b2 = p[o:o + h]; o += h
    W3 = p[o:o + k * h].reshape(k, h); o += k * h
    b3 = p[o:o + k]; o += k
    assert o == p.size
    return W1, b1, W2, b2, W3, b3


def forward(p, X):
    """Predictions [n, K] for inputs X [n, D]."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.tanh(X @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    return h2 @ W3.T + b3


def loss(p, X, T):
    Y = forward(p, X)
    T = np.asarray(T, dtype=np.float64)
    return 0.5 * np.sum((Y - T) ** 2) / X.shape[0]


def grad(p, X, T):
    """Backpropagation of the loss above: returns dL/dp packed like p."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    n = X.shape[0]
    h1 = np.tanh(X @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    Y = h2 @ W3.T + b3
    dY = (Y - T) / n                      # dL/dY
    gW3 = dY.T @ h2
    gb3 = dY.sum(axis=0)
    dh2 = dY @ W3                         # dL/dh2
    dz2 = dh2 * (1.0 - h2 ** 2)           # tanh'
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(axis=0)
    dh1 = dz2 @ W2
    dz1 = dh1 * (1.0 - h1 ** 2)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(axis=0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])


def sgd_step(p, X, T, lr):
    return np.asarray(p, dtype=np.float64) - lr * grad(p, X, T)


def init_params(seed: int, scale: float = 0.5) -> np.ndarray:
    """Deterministic initial weights (uniform in [-scale/sqrt(fan_in), +...]); biases 0."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_out, fan_in in ((H, D), (H, H), (K, H)):
        lim = scale / np.sqrt(fan_in)
        parts.append(rng.uniform(-lim, lim, size=fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts)
