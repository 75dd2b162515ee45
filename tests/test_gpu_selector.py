"""GPU parity of the learned exchange selector's kernels against the CPU MLP
oracle, and invariance of results when the selector drives the exchange."""
import numpy as np
import pytest

import graphgen
import oracle
from oracle import mlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ipg():
    import paper_2010_08781_amd as m

    m.lib()
    return m


def _batch(n, seed):
    rng = np.random.default_rng(seed)
    X = np.stack([rng.uniform(0, 1, n), rng.uniform(0, 1, n), rng.uniform(0, 2, n), rng.uniform(0.3, 1, n)], axis=1)
    T = np.stack([8 * X[:, 1] - 3 * X[:, 0] + 4, 2 + 6 * X[:, 3] - X[:, 2], 5 * X[:, 0] * X[:, 3] + 1], axis=1)
    return X, T


def _cuda(a):
    import torch

    return torch.tensor(a, dtype=torch.float64, device="cuda")


def test_forward_matches_oracle(ipg):
    X, _ = _batch(1000, 1)
    p = mlp.init_params(4, scale=2.0)
    y = ipg.selector_forward(_cuda(p), _cuda(X)).cpu().numpy()
    np.testing.assert_allclose(y, mlp.forward(p, X), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("n", [1, 37, 700])
def test_grad_matches_oracle(ipg, n):
    X, T = _batch(n, 2)
    p = mlp.init_params(5, scale=2.0)
    g = ipg.selector_grad(_cuda(p), _cuda(X), _cuda(T)).cpu().numpy()
    ref = mlp.grad(p, X, T)
    assert np.max(np.abs(g - ref)) <= 1e-11 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("epochs,tol", [(5, 1e-12), (200, 1e-5)])
def test_train_matches_oracle_and_descends(ipg, epochs, tol):
    # Each step agrees to rounding (see the gradient test); over many steps
    # the last-bit differences of summation order and tanh are amplified by
    # the iteration, hence the looser bound on the long trajectory.
    X, T = _batch(300, 3)
    p0 = mlp.init_params(6)
    pt = _cuda(p0)
    ipg.selector_train(pt, _cuda(X), _cuda(T), epochs=epochs, lr=0.05)
    ref = p0.copy()
    for _ in range(epochs):
        ref = mlp.sgd_step(ref, X, T, 0.05)
    got = pt.cpu().numpy()
    assert np.max(np.abs(got - ref)) <= tol
    if epochs >= 200:
        assert mlp.loss(got, X, T) < 0.5 * mlp.loss(p0, X, T)


def test_features_definition(ipg):
    x = ipg.selector_features([0, 1023], [0, 4095], [0, 500], 2 ** 20 - 1)
    np.testing.assert_allclose(x, [[0, 0, 0, 20 / 32], [10 / 32, 12 / 32, 2.0, 20 / 32]])


@pytest.mark.parametrize("app", ["cc", "sssp"])
def test_selector_never_changes_results(ipg, app):
    # Two selectors that always prefer push or always pull (output biases),
    # and a random one: values and traces equal the oracle's, and the
    # exchange actually follows the network.
    hg = graphgen.rmat(14, 16, seed=3, symmetric=True)
    ref = oracle.run_graph(app, hg, 0, source=0)
    g = ipg.Graph.from_host(hg)
    always_push = np.zeros(mlp.n_params())
    always_push[-3:] = [0.0, 0.0, 1.0]  # push (over the list when there is one), never pull
    always_pull = np.zeros(mlp.n_params())
    always_pull[-3:] = [1.0, 1.0, 0.0]
    for p, want in ((always_push, 1), (always_pull, 2), (mlp.init_params(9, scale=3.0), None)):
        # without the late push, which may turn a chosen pull into a push once the messages are counted
        vals, st = g.run(app, source=0, selector=_cuda(p), tuning={"late_div": 0xFFFFFFFF})
        assert np.array_equal(ipg.values_to_numpy(vals), ref.values)
        assert np.array_equal(st.trace, ref.trace)
        if want is not None:
            assert set(st.mode.tolist()) == {want}
