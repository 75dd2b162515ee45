"""Pins for the selector MLP oracle: finite differences, autograd, descent."""
import numpy as np
import torch

from oracle import mlp


def _data(n=40, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, size=(n, mlp.D))
    T = np.stack([np.sin(2 * X[:, 0]) + X[:, 1] * X[:, 3], X[:, 2] ** 2 - X[:, 0], np.cos(X[:, 1]) * X[:, 2]], axis=1)
    return X, T


def test_param_count():
    assert mlp.n_params() == 16 * 4 + 16 + 16 * 16 + 16 + 3 * 16 + 3 == 403
    assert mlp.init_params(1).size == mlp.n_params()


def test_grad_matches_central_differences():
    X, T = _data()
    p = mlp.init_params(3, scale=1.5)
    g = mlp.grad(p, X, T)
    eps = 1e-6
    num = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = eps
        num[i] = (mlp.loss(p + e, X, T) - mlp.loss(p - e, X, T)) / (2 * eps)
    assert np.max(np.abs(num - g)) <= 1e-8 * max(1.0, np.max(np.abs(g)))


def test_grad_matches_torch_autograd_float64():
    X, T = _data(n=33, seed=5)
    p = mlp.init_params(7, scale=2.0)
    W1, b1, W2, b2, W3, b3 = [torch.tensor(a.copy(), dtype=torch.float64, requires_grad=True) for a in mlp.unpack(p)]
    x = torch.tensor(X)
    y = torch.tanh(torch.tanh(x @ W1.T + b1) @ W2.T + b2) @ W3.T + b3
    L = 0.5 * ((y - torch.tensor(T)) ** 2).sum() / X.shape[0]
    L.backward()
    ref = np.concatenate([t.grad.numpy().ravel() for t in (W1, b1, W2, b2, W3, b3)])
    np.testing.assert_allclose(mlp.grad(p, X, T), ref, rtol=1e-12, atol=1e-14)
    assert abs(float(L) - mlp.loss(p, X, T)) <= 1e-14


def test_forward_zero_hidden_is_output_bias():
    p = np.zeros(mlp.n_params())
    p[-3:] = [0.25, -3.0, 1.5]
    X, _ = _data(n=5)
    np.testing.assert_array_equal(mlp.forward(p, X), np.tile([0.25, -3.0, 1.5], (5, 1)))


def test_sgd_descends():
    X, T = _data(n=64, seed=2)
    p = mlp.init_params(11)
    l0 = mlp.loss(p, X, T)
    for _ in range(300):
        p = mlp.sgd_step(p, X, T, 0.1)
    assert mlp.loss(p, X, T) < 0.5 * l0
