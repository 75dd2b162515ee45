"""The oracle's pull form (Section 4.3.2) under an OpenMP static schedule
(Section 4.2): its output must not depend on the thread count, and must equal
the push form's -- bit for bit, values and trace -- when every CSC list is
sorted by source (the same messages combined in the same order).  With the
lists in another order the minima stay bit-exact and PageRank moves only by
rounding.  Errors (cap, overflow, bad source) come out as in the push form."""
import numpy as np
import pytest

import graphgen
import oracle
from tests.graphs_small import path, random_graph


def _cases():
    yield "rmat14-dir", graphgen.rmat(14, 16, seed=1)
    yield "rmat12-sym", graphgen.rmat(12, 16, seed=2, symmetric=True)
    yield "multi-loops", random_graph(500, 4000, seed=5, loops=True, dups=True)
    yield "multi-sym-w", random_graph(400, 3000, seed=6, symmetric=True, loops=True, dups=True, weight_seed=7)
    yield "grid64", graphgen.grid_with_shortcuts(64, 0.01, seed=3)


CASES = list(_cases())


def _runs(g):
    yield "pagerank", 10, 0
    yield "cc", 0, 0
    yield "sssp", 0, 0
    yield "sssp", 0, int(g.n // 3)


@pytest.mark.parametrize("name,g", CASES, ids=[c[0] for c in CASES])
def test_pull_equals_push_bitwise_and_any_thread_count(name, g):
    for app, param, src in _runs(g):
        push = oracle.run_graph(app, g, param, source=src)
        one = oracle.run_pull(app, g, param, source=src, threads=1)
        many = oracle.run_pull(app, g, param, source=src, threads=8)
        dealt = oracle.run_pull(app, g, param, source=src, threads=5, chunk=7)
        assert dealt.values.tobytes() == many.values.tobytes() and np.array_equal(dealt.trace, many.trace)
        assert push.status == one.status == many.status == oracle.OK, (app, src)
        assert push.supersteps == one.supersteps == many.supersteps
        # bit for bit (PageRank too: same additions in the same order)
        assert one.values.tobytes() == many.values.tobytes(), (app, src)
        assert push.values.tobytes() == one.values.tobytes(), (app, src)
        assert np.array_equal(push.trace, one.trace) and np.array_equal(one.trace, many.trace), (app, src)


def test_pull_damping_matches_push():
    g = graphgen.rmat(12, 16, seed=8)
    for d in (0.5, 0.9):
        a = oracle.run_graph("pagerank", g, 7, damping=d)
        b = oracle.run_pull("pagerank", g, 7, damping=d, threads=4)
        assert a.values.tobytes() == b.values.tobytes()


def _shuffled_csc(g, seed):
    """The same graph with every CSC list (and its weights) in a random order."""
    rng = np.random.default_rng(seed)
    src = g.csc_src.copy()
    w = None if g.csc_w is None else g.csc_w.copy()
    for v in range(g.n):
        a, b = int(g.csc_off[v]), int(g.csc_off[v + 1])
        p = rng.permutation(b - a) + a
        src[a:b] = g.csc_src[p]
        if w is not None:
            w[a:b] = g.csc_w[p]
    return graphgen.HostGraph(n=g.n, csr_off=g.csr_off, csr_dst=g.csr_dst, csc_off=g.csc_off, csc_src=src,
                              csr_w=g.csr_w, csc_w=w)


def test_pull_unsorted_lists():
    g = _shuffled_csc(random_graph(600, 5000, seed=11, loops=True, dups=True, weight_seed=4), seed=1)
    for app in ("cc", "sssp"):
        a = oracle.run_graph(app, g, 0)
        b = oracle.run_pull(app, g, 0, threads=3)
        assert np.array_equal(a.values, b.values) and np.array_equal(a.trace, b.trace)
    a = oracle.run_graph("pagerank", g, 10)
    b = oracle.run_pull("pagerank", g, 10, threads=3)
    np.testing.assert_allclose(b.values, a.values, rtol=1e-13, atol=0)
    assert np.array_equal(a.trace, b.trace)


def test_pull_cap_overflow_and_source():
    g = path(40)
    a = oracle.run_graph("cc", g, 5)
    b = oracle.run_pull("cc", g, 5, threads=2)
    assert a.status == b.status == oracle.NOT_CONVERGED
    assert a.supersteps == b.supersteps == 5
    assert np.array_equal(a.values, b.values) and np.array_equal(a.trace, b.trace)
    # weights that reach INF on the third hop: overflow in the same superstep
    src, dst = np.arange(3), np.arange(1, 4)
    big = graphgen.from_edges(4, src, dst, symmetric=True, weight_seed=1)
    big.csr_w[:] = 0x7FFFFFFF
    a = oracle.run_graph("sssp", big, 0)
    b = oracle.run_pull("sssp", big, 0, threads=2)
    assert a.status == b.status == oracle.EOVERFLOW
    assert a.supersteps == b.supersteps
    assert oracle.run_pull("sssp", g, 0, source=g.n).status == oracle.EINVAL


def test_pull_empty_and_single_vertex():
    e = graphgen.from_edges(5, [], [])
    for app, param in (("pagerank", 3), ("cc", 0), ("sssp", 0)):
        a = oracle.run_graph(app, e, param)
        b = oracle.run_pull(app, e, param, threads=4)
        assert a.status == b.status == oracle.OK
        assert a.values.tobytes() == b.values.tobytes() and np.array_equal(a.trace, b.trace)
