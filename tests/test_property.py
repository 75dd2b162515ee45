"""Property-based pins of the oracle on random small graphs (hypothesis):
hash-min CC against union-find components, SSSP against scipy's Dijkstra,
PageRank's rank-sum balance and teleport floor, and the pull form under
OpenMP equal to the sequential push form bit for bit (sorted lists)."""
import numpy as np
import pytest
import scipy.sparse as sp
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st
from scipy.sparse import csgraph

import oracle
from tests.graph_strategies import small_graphs
from tests.graphs_small import edge_arrays

SETTINGS = settings(max_examples=150, deadline=None, derandomize=True,
                    suppress_health_check=[HealthCheck.too_slow, HealthCheck.data_too_large])


@SETTINGS
@given(small_graphs())
def test_cc_is_min_id_of_reaching_component(g):
    r = oracle.run_graph("cc", g, 0)
    assert r.status == oracle.OK
    s, d = edge_arrays(g)
    A = sp.csr_matrix((np.ones(s.size), (s, d)), shape=(g.n, g.n))
    if g.symmetric:
        _, lab = csgraph.connected_components(A, directed=False)
        want = np.array([np.flatnonzero(lab == lab[v]).min() for v in range(g.n)], dtype=np.uint32)
    else:  # min id among the vertices with a path to v (v included)
        reach = csgraph.shortest_path(A, unweighted=True) < np.inf
        want = np.array([np.flatnonzero(reach[:, v]).min() for v in range(g.n)], dtype=np.uint32)
    assert np.array_equal(r.values, want)


@SETTINGS
@given(small_graphs())
def test_sssp_is_dijkstra(g):
    src = 0
    r = oracle.run_graph("sssp", g, 0, source=src)
    assert r.status == oracle.OK
    s, d = edge_arrays(g)
    w = g.csr_w.astype(np.float64) if g.csr_w is not None else np.ones(s.size)
    # the lightest of duplicate edges is the one that counts
    best = {}
    for a, b, x in zip(s.tolist(), d.tolist(), w.tolist()):
        best[(a, b)] = min(best.get((a, b), np.inf), x)
    if best:
        k = np.array(list(best.keys()))
        A = sp.csr_matrix((np.array(list(best.values())), (k[:, 0], k[:, 1])), shape=(g.n, g.n))
    else:
        A = sp.csr_matrix((g.n, g.n))
    dist = csgraph.dijkstra(A, indices=src)
    want = np.where(np.isinf(dist), oracle.INF, dist).astype(np.uint64).astype(np.uint32)
    assert np.array_equal(r.values, want)


@SETTINGS
@given(small_graphs(weighted=False), st.integers(1, 12), st.sampled_from([0.85, 0.5, 0.99]))
def test_pagerank_balance_and_teleport_floor(g, T, d):
    prev = oracle.run_graph("pagerank", g, T - 1, damping=d).values
    cur = oracle.run_graph("pagerank", g, T, damping=d)
    assert cur.status == oracle.OK and cur.supersteps == T + 1
    dangling = np.diff(g.csr_off) == 0
    expect = (1.0 - d) + d * (prev.sum() - prev[dangling].sum())
    assert abs(cur.values.sum() - expect) <= 1e-13
    assert np.all(cur.values >= (1.0 - d) / g.n)
    noin = np.diff(g.csc_off) == 0
    assert np.all(cur.values[noin] == (1.0 - d) / g.n)


@SETTINGS
@given(small_graphs())
def test_pull_form_equals_push_form(g):
    for app, param in (("pagerank", 7), ("cc", 0), ("sssp", 0)):
        a = oracle.run_graph(app, g, param)
        b = oracle.run_pull(app, g, param, threads=3, chunk=2)
        assert a.status == b.status
        assert a.values.tobytes() == b.values.tobytes(), app
        assert np.array_equal(a.trace, b.trace), app
