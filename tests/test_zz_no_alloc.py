"""The allocation-free selector training entry point against the one that
takes a workspace: same parameters bit for bit, on two calls in a row (the
second with fewer samples, so that it runs over what the first left in the
library's scratch array), and the size limit."""

import numpy as np
import pytest

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


def test_noalloc_train_matches_workspace_train(ipg):
    import torch

    from oracle import mlp

    dev = torch.device("cuda")
    p0 = torch.tensor(mlp.init_params(7, scale=1.0), dtype=torch.float64, device=dev)
    for n, epochs, seed in ((3000, 40, 11), (700, 25, 12)):
        X, T = _batch(n, seed)
        x = torch.tensor(X, dtype=torch.float64, device=dev)
        t = torch.tensor(T, dtype=torch.float64, device=dev)
        a = p0.clone()
        b = p0.clone()
        ipg.selector_train(a, x, t, epochs, 0.05)
        ipg.selector_train_noalloc(b, x, t, epochs, 0.05)
        torch.cuda.synchronize()
        assert torch.equal(a, b), f"n={n}: parameters differ"
        assert not torch.equal(a, p0)


def test_noalloc_train_limit(ipg):
    import torch

    n = ipg.SELECTOR_NOALLOC_MAX_SAMPLES + 1
    x = torch.zeros((n, 4), dtype=torch.float64, device="cuda")
    t = torch.zeros((n, ipg.SELECTOR_OUTPUTS), dtype=torch.float64, device="cuda")
    p = torch.zeros(ipg.SELECTOR_PARAMS, dtype=torch.float64, device="cuda")
    rc = ipg.lib().ipg_selector_train_noalloc(p.data_ptr(), x.data_ptr(), t.data_ptr(), n, 1, 0.1, None)
    assert rc == -1  # IPG_EINVAL
    assert b"IPG_SELECTOR_NOALLOC_MAX_SAMPLES" in ipg.lib().ipg_last_error()
