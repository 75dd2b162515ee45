"""GPU parity of PageRank run to convergence (L1 change below a tolerance).

The stopping update must be the oracle's, the ranks those of the oracle's
fixed-length run with that many updates (within the PageRank tolerance), and
the reported per-update changes the oracle's.  Tolerances are placed away
from every change of the run, so that summation order cannot move the stop.
"""
import numpy as np
import pytest

import graphgen
import oracle
from tests.graphs_small import random_graph

pytestmark = pytest.mark.gpu

PR_RTOL = 1e-12


@pytest.fixture(scope="module")
def ipg():
    import torch

    import paper_2010_08781_amd as m

    assert torch.cuda.is_available()
    m.lib()
    return m


# The GPU ranks differ from the oracle's by a few ulps (another summation
# order), so a change reported by the GPU differs from the oracle's by up to
# about N ulps of a rank: about 1e-14 absolute, with ranks summing to <= 1.
DELTA_ATOL = 1e-13


def clear_tol(d, tol):
    """Move tol until no change of the run lies within reach of that noise."""
    while np.any(np.abs(d[1:] - tol) <= max(1e-6 * tol, 10 * DELTA_ATOL)):
        tol *= 1.37
    return tol


@pytest.mark.parametrize("hg_name", ["rmat-s14-dir", "random-sym"])
def test_converges_at_the_oracles_update(ipg, hg_name):
    hg = graphgen.workload(hg_name) if hg_name.startswith("rmat") else random_graph(5000, 40000, seed=3, symmetric=True)
    g = ipg.Graph.from_host(hg)
    Tmax = 120
    d = oracle.pagerank_deltas(hg.n, hg.csr_off, hg.csr_dst, Tmax)
    for tol in (1e-3, 1e-6, 1e-9):
        tol = clear_tol(d, tol)
        ref, T, _ = oracle.pagerank_converge(hg, tol, Tmax)
        assert T < Tmax
        for mode in ("pull", "push"):
            r, st = g.run("pagerank", Tmax, mode=mode, tol=tol)
            assert st.status == ipg.OK and st.halted
            assert st.supersteps == T + 1, (mode, tol, st.supersteps, T + 1)
            err = float(np.max(np.abs(r.cpu().numpy() - ref.values) / ref.values))
            assert err <= PR_RTOL, (mode, tol, err)
            np.testing.assert_allclose(st.residual[1:], d[1: T + 1], rtol=1e-9, atol=DELTA_ATOL)
            assert np.array_equal(st.trace, ref.trace)


def test_cap_before_convergence(ipg):
    hg = random_graph(3000, 20000, seed=4)
    g = ipg.Graph.from_host(hg)
    ref = oracle.run_graph("pagerank", hg, 6)
    for mode in ("pull", "push"):
        r, st = g.run("pagerank", 6, mode=mode, tol=1e-300)
        assert st.status == ipg.NOT_CONVERGED and not st.halted and st.supersteps == 7
        assert float(np.max(np.abs(r.cpu().numpy() - ref.values) / ref.values)) <= PR_RTOL


def test_parts_converge_consistently(ipg):
    # over a disjoint union the change is summed over all parts; the result
    # is the fixed-length run with the same parts and the stopping T
    import torch

    graphs = [graphgen.rmat_small(n, 8, seed=500 + n) for n in (1500, 4000, 900)]
    u = graphgen.disjoint_union(graphs)
    g = ipg.Graph.from_host(u)
    parts = torch.from_numpy(u.meta["parts"].astype(np.int32)).cuda()
    r, st = g.run("pagerank", 200, parts=parts, tol=1e-9)
    assert st.status == ipg.OK
    T = st.supersteps - 1
    fixed, _ = g.run("pagerank", T, parts=parts)
    assert torch.equal(r, fixed)
    assert st.residual[T] < 1e-9 <= st.residual[T - 1]


def test_tolerance_errors(ipg):
    hg = random_graph(100, 300, seed=1)
    g = ipg.Graph.from_host(hg)
    for kw, status in ((dict(app="cc", tol=1e-6), ipg.EUNSUPPORTED),
                       (dict(app="pagerank", tol=-1.0, max_supersteps=5), ipg.EINVAL),
                       (dict(app="pagerank", tol=1e-6, max_supersteps=0), ipg.EINVAL),
                       (dict(app="pagerank", tol=1e-6, max_supersteps=5, graph=True), ipg.EUNSUPPORTED)):
        with pytest.raises(ipg.IpgError) as e:
            g.run(**kw)
        assert e.value.status == status, kw
