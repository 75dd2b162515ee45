"""Pins for the CPU oracle: closed forms, invariants and textbook routines.

Each test checks the oracle against something other than itself -- a value
fixed by mathematics, an independent formulation (dense or sparse linear
algebra, exact rationals), or a library routine (scipy's BFS, Dijkstra and
connected components) -- chosen so that a plausible slip (a dropped term, a
wrong constant, a transposed operand, a lost BSP barrier) fails one of them.
"""
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse import csgraph

import graphgen
import oracle
from tests.graphs_small import (complete_digraph, directed_cycle, edge_arrays, path, random_graph,
                                strongly_connected_random)

INF = oracle.INF


def pr(g, T):
    r = oracle.run_graph("pagerank", g, T)
    assert r.status == oracle.OK
    assert r.supersteps == T + 1
    return r


def adjacency(g):
    """Sparse A with A[u, v] = number of edges u -> v (duplicates counted)."""
    s, d = edge_arrays(g)
    return sp.csr_matrix((np.ones(s.size), (s, d)), shape=(g.n, g.n))


# ---------------------------------------------------------------- PageRank --

@pytest.mark.parametrize("n", [1, 2, 7, 64, 1000])
def test_pr_directed_cycle_is_uniform(n):
    # Fig. 8 on a directed cycle: every vertex has in = out = 1, so 1/N is a
    # fixed point of r <- 0.15/N + 0.85 r; all updates stay at 1/N.
    g = directed_cycle(n) if n > 1 else graphgen.from_edges(1, [0], [0], keep_self_loops=True)
    for T in range(0, 11):
        r = pr(g, T)
        np.testing.assert_allclose(r.values, 1.0 / n, rtol=4e-16 * (T + 1), atol=0)


@pytest.mark.parametrize("n", [2, 5, 17])
def test_pr_complete_digraph_is_uniform(n):
    g = complete_digraph(n)
    for T in (1, 2, 10):
        np.testing.assert_allclose(pr(g, T).values, 1.0 / n, rtol=1e-14, atol=0)


@pytest.mark.parametrize("d", [0.85, 0.5, 0.3])
def test_pr_source_only_vertices_get_exactly_the_teleport_term(d):
    # A vertex without in-edges receives no message: after any update its rank
    # is exactly the teleport term (1-d)/N (the sum is 0.0), and no other
    # vertex's is below it.
    g = random_graph(300, 900, seed=3)
    indeg = np.diff(g.csc_off)
    assert (indeg == 0).any()
    for T in (1, 3, 10):
        r = oracle.run_graph("pagerank", g, T, damping=d)
        assert r.status == oracle.OK
        assert np.all(r.values[indeg == 0] == (1.0 - d) / g.n)
        assert np.all(r.values[indeg > 0] > (1.0 - d) / g.n)


def test_pr_T0_is_initial_value():
    g = random_graph(50, 200, seed=1)
    r = pr(g, 0)
    assert np.all(r.values == 1.0 / 50)
    assert r.trace.tolist() == [[50, 0, 0]]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_pr_rank_mass_balance(seed):
    # Sum over v of r_{k+1}(v) = 0.15 + 0.85 * (sum r_k - sum of dangling r_k):
    # every non-dangling vertex passes all its mass on, dangling mass is lost.
    g = random_graph(500, 2000, seed=seed)
    dangling = np.diff(g.csr_off) == 0
    assert dangling.any()
    prev = pr(g, 0).values
    for T in range(1, 11):
        cur = pr(g, T).values
        expect = 0.15 + 0.85 * (prev.sum() - prev[dangling].sum())
        assert abs(cur.sum() - expect) <= 1e-12
        prev = cur


def test_pr_mass_conserved_without_dangling():
    g = strongly_connected_random(400, 1600, seed=5)
    assert (np.diff(g.csr_off) > 0).all()
    for T in (1, 5, 10):
        assert abs(pr(g, T).values.sum() - 1.0) <= 1e-13


def _pr_matrix_form(g, T):
    # Second, independent formulation (the matrix form of Ligra's listing in
    # Fig. 16 / Pregel's Fig. 12): r <- 0.15/N + 0.85 * A^T (D^+ r), where
    # D^+ inverts the out-degree and is 0 for dangling vertices.
    A = adjacency(g)
    deg = np.asarray(A.sum(axis=1)).ravel()
    dinv = np.where(deg > 0, 1.0 / np.where(deg > 0, deg, 1), 0.0)
    At = A.T.tocsr()
    r = np.full(g.n, 1.0 / g.n)
    for _ in range(T):
        r = 0.15 / g.n + 0.85 * (At @ (dinv * r))
    return r


@pytest.mark.parametrize("case", ["rand", "loops_dups", "rmat10"])
def test_pr_matches_matrix_form(case):
    if case == "rand":
        g = random_graph(700, 5000, seed=11)
    elif case == "loops_dups":
        g = random_graph(200, 1500, seed=12, loops=True, dups=True)
    else:
        g = graphgen.rmat(10, 16, seed=9)
    for T in (1, 2, 5, 10):
        ref = _pr_matrix_form(g, T)
        got = pr(g, T).values
        assert np.max(np.abs(got - ref) / ref) <= 1e-13


def test_pr_rmat_s14_matches_sparse_matrix_form():
    # the small parity workload: R-MAT scale 14, edge factor 16, seed 1.
    g = graphgen.workload("rmat-s14-dir")
    ref = _pr_matrix_form(g, 10)
    got = pr(g, 10).values
    assert np.max(np.abs(got - ref) / ref) <= 1e-12


@pytest.mark.parametrize("seed", [21, 22])
def test_pr_converges_to_linear_fixed_point(seed):
    # Closed form: for T -> infinity the iteration reaches the unique solution
    # of (I - 0.85 A^T D^+) r = 0.15/N * 1; the error contracts by 0.85 per
    # update, so after 250 updates it is below 1e-15 relative.
    g = random_graph(60, 240, seed=seed)
    A = adjacency(g).toarray()
    deg = A.sum(axis=1)
    dinv = np.where(deg > 0, 1.0 / np.where(deg > 0, deg, 1), 0.0)
    M = np.eye(g.n) - 0.85 * (A.T * dinv[None, :])
    exact = np.linalg.solve(M, np.full(g.n, 0.15 / g.n))
    got = pr(g, 250).values
    assert np.max(np.abs(got - exact) / exact) <= 1e-12


def test_pr_exact_rationals_small():
    # The exact rational iterate (3/20 for 0.15, 17/20 for 0.85) computed in
    # matrix form; the oracle's doubles must agree within 1e-14.
    g = random_graph(40, 160, seed=31, loops=True, dups=True)
    n = g.n
    s, d = edge_arrays(g)
    deg = np.bincount(s, minlength=n)
    r = [Fraction(1, n)] * n
    for _ in range(10):
        acc = [Fraction(0)] * n
        for u, v in zip(s.tolist(), d.tolist()):
            acc[v] += r[u] / int(deg[u])
        r = [Fraction(3, 20) / n + Fraction(17, 20) * a for a in acc]
    got = pr(g, 10).values
    exact = np.array([float(x) for x in r])
    assert np.max(np.abs(got - exact) / exact) <= 1e-14


def test_pr_trace_counts():
    g = random_graph(100, 400, seed=2)
    r = pr(g, 10)
    dang = int((np.diff(g.csr_off) == 0).sum())
    assert r.trace[:, 0].tolist() == [100] * 11
    assert r.trace[:, 1].tolist() == [100] * 10 + [0]
    assert r.trace[:, 2].tolist() == [g.m] * 10 + [0]
    assert dang > 0  # dangling vertices broadcast to nobody yet count as broadcasting


# --------------------------------------------------------------------- CC --

def _components_min_label(g):
    ncomp, lab = csgraph.connected_components(adjacency(g), directed=False)
    mins = np.full(ncomp, np.iinfo(np.int64).max)
    np.minimum.at(mins, lab, np.arange(g.n))
    return mins[lab].astype(np.uint32)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_cc_matches_union_find(seed):
    g = random_graph(2000, 1500 + 500 * seed, seed=seed, symmetric=True)
    r = oracle.run_graph("cc", g, 0)
    assert r.status == oracle.OK
    np.testing.assert_array_equal(r.values, _components_min_label(g))


def test_cc_rmat_s14_symmetrised_matches_union_find():
    g = graphgen.rmat(14, 16, seed=1, symmetric=True)
    r = oracle.run_graph("cc", g, 0)
    np.testing.assert_array_equal(r.values, _components_min_label(g))


def test_cc_directed_is_min_reaching_id():
    # On a directed graph the label is the minimum id among vertices with a
    # path to the vertex (itself included): brute force by BFS from every id.
    g = random_graph(60, 90, seed=7)
    A = adjacency(g)
    reach = csgraph.shortest_path(A, unweighted=True, directed=True) < np.inf  # reach[u, v]: u ->* v
    expect = np.array([np.flatnonzero(reach[:, v]).min() for v in range(g.n)], dtype=np.uint32)
    np.testing.assert_array_equal(oracle.run_graph("cc", g, 0).values, expect)


def test_cc_empty_graph_one_superstep():
    g = graphgen.from_edges(5, [], [])
    r = oracle.run_graph("cc", g, 0)
    assert r.supersteps == 1 and r.values.tolist() == [0, 1, 2, 3, 4]
    assert r.trace.tolist() == [[5, 5, 0]]


@pytest.mark.parametrize("n", [2, 3, 4, 9])
def test_cc_path_superstep_count(n):
    # Label 0 advances one hop per superstep: vertex n-1 gets it in superstep
    # n-1 and echoes it back, which changes nothing in superstep n.
    r = oracle.run_graph("cc", path(n), 0)
    assert r.supersteps == n + 1
    assert r.values.tolist() == [0] * n


def test_cc_path3_trace_by_hand():
    # Hand-derived from Fig. 9 on the undirected path 0-1-2 (degrees 1, 2, 1):
    # s0 all send (4 messages); s1 vertices 1 and 2 lower their label and send
    # 2 + 1 messages; s2 only vertex 2 lowers (to 0) and sends 1; s3 vertex 1
    # receives 0, changes nothing.
    r = oracle.run_graph("cc", path(3), 0)
    assert r.trace.tolist() == [[3, 3, 4], [3, 2, 3], [3, 1, 1], [1, 0, 0]]


def test_cc_cap_reports_not_converged():
    r = oracle.run_graph("cc", path(9), 3)
    assert r.status == oracle.NOT_CONVERGED and r.supersteps == 3


# ------------------------------------------------------------------- SSSP --

def _bfs_levels(g, src):
    d = csgraph.shortest_path(adjacency(g), unweighted=True, directed=True, indices=src)
    return np.where(np.isinf(d), INF, d).astype(np.uint32)


@pytest.mark.parametrize("sym", [False, True])
@pytest.mark.parametrize("seed", [0, 1])
def test_sssp_unweighted_matches_bfs(sym, seed):
    g = random_graph(3000, 6000, seed=seed, symmetric=sym)
    for src in (0, 17, 2999):
        r = oracle.run_graph("sssp", g, 0, source=src, weighted=False)
        assert r.status == oracle.OK
        np.testing.assert_array_equal(r.values, _bfs_levels(g, src))


def test_sssp_rmat_s14_matches_bfs():
    g = graphgen.rmat(14, 16, seed=1, symmetric=True)
    r = oracle.run_graph("sssp", g, 0, source=0)
    np.testing.assert_array_equal(r.values, _bfs_levels(g, 0))


@pytest.mark.parametrize("sym", [False, True])
def test_sssp_weighted_matches_dijkstra(sym):
    g = random_graph(2000, 8000, seed=5, symmetric=sym, weight_seed=77)
    s, d = edge_arrays(g)
    A = sp.csr_matrix((g.csr_w.astype(np.float64), (s, d)), shape=(g.n, g.n))
    for src in (0, 5):
        ref = csgraph.dijkstra(A, directed=True, indices=src)
        ref = np.where(np.isinf(ref), INF, ref).astype(np.uint32)
        r = oracle.run_graph("sssp", g, 0, source=src)
        np.testing.assert_array_equal(r.values, ref)


def test_sssp_weighted_tiny_floyd_warshall():
    # Brute force on a tiny multigraph with self-loops: Floyd-Warshall with
    # the minimum weight over parallel edges.
    g = random_graph(12, 40, seed=9, loops=True, dups=True, weight_seed=5)
    s, d = edge_arrays(g)
    D = np.full((g.n, g.n), np.inf)
    np.fill_diagonal(D, 0)
    for u, v, w in zip(s, d, g.csr_w):
        D[u, v] = min(D[u, v], float(w)) if u != v else 0
    for k in range(g.n):
        D = np.minimum(D, D[:, [k]] + D[[k], :])
    for src in range(g.n):
        r = oracle.run_graph("sssp", g, 0, source=src)
        np.testing.assert_array_equal(r.values, np.where(np.isinf(D[src]), INF, D[src]).astype(np.uint32))


def test_sssp_grid_weighted_matches_dijkstra():
    g = graphgen.grid_with_shortcuts(64, 0.01, seed=3)
    s, d = edge_arrays(g)
    A = sp.csr_matrix((g.csr_w.astype(np.float64), (s, d)), shape=(g.n, g.n))
    ref = csgraph.dijkstra(A, directed=True, indices=0).astype(np.uint32)
    np.testing.assert_array_equal(oracle.run_graph("sssp", g, 0, source=0).values, ref)


def test_sssp_superstep_counts_by_hand():
    # Directed path 0->1->2: s0 source sends, s1 vertex 1 relays, s2 vertex 2
    # updates and broadcasts to nobody -> 3 supersteps.  Undirected: vertex 2
    # also messages vertex 1 back, which changes nothing in s3 -> 4.
    r = oracle.run_graph("sssp", path(3, directed=True), 0, source=0)
    assert r.supersteps == 3 and r.values.tolist() == [0, 1, 2]
    assert r.trace.tolist() == [[3, 1, 1], [1, 1, 1], [1, 1, 0]]
    r = oracle.run_graph("sssp", path(3), 0, source=0)
    assert r.supersteps == 4 and r.values.tolist() == [0, 1, 2]


def test_sssp_unreachable_stays_inf_and_source_checked():
    g = graphgen.from_edges(4, [0, 2], [1, 3])
    r = oracle.run_graph("sssp", g, 0, source=0)
    assert r.values.tolist() == [0, 1, INF, INF]
    assert oracle.run_graph("sssp", g, 0, source=4).status == oracle.EINVAL


def test_sssp_overflow_is_an_error():
    g = graphgen.from_edges(3, [0, 1], [1, 2])
    w = np.array([0xFFFFFFF0, 0x20], dtype=np.uint32)
    r = oracle.run("sssp", 3, g.csr_off, g.csr_dst, 0, source=0, csr_w=w)
    assert r.status == oracle.EOVERFLOW


def test_bad_graph_rejected():
    off = np.array([0, 2, 1], dtype=np.uint64)
    assert oracle.run("cc", 2, off, np.array([1, 0], np.int32), 0).status == oracle.EBADGRAPH
    off = np.array([0, 1, 2], dtype=np.uint64)
    assert oracle.run("cc", 2, off, np.array([1, 2], np.int32), 0).status == oracle.EBADGRAPH


# ----------------------------------------------- PageRank to convergence --

def test_pr_deltas_exact_rationals():
    # The L1 change of every update, from the exact rational iterates
    # (3/20, 17/20), against the oracle's doubles.
    g = random_graph(30, 120, seed=44, loops=True, dups=True)
    n = g.n
    s, d = edge_arrays(g)
    deg = np.bincount(s, minlength=n)
    r = [Fraction(1, n)] * n
    exact = [Fraction(0)]
    for _ in range(12):
        acc = [Fraction(0)] * n
        for u, v in zip(s.tolist(), d.tolist()):
            acc[v] += r[u] / int(deg[u])
        nr = [Fraction(3, 20) / n + Fraction(17, 20) * a for a in acc]
        exact.append(sum(abs(a - b) for a, b in zip(nr, r)))
        r = nr
    got = oracle.pagerank_deltas(n, g.csr_off, g.csr_dst, 12)
    ex = np.array([float(x) for x in exact])
    assert got[0] == 0.0
    assert np.all(np.abs(got[1:] - ex[1:]) <= 1e-13 * ex[1:] + 1e-18)


def test_pr_deltas_contract_by_damping():
    # r' = 0.15/N + 0.85 M r with column sums of M at most 1 (dangling mass is
    # dropped), so ||r_{s+1} - r_s||_1 <= 0.85 ||r_s - r_{s-1}||_1.
    for seed in (1, 2, 3):
        g = random_graph(500, 3000, seed=seed)
        d = oracle.pagerank_deltas(g.n, g.csr_off, g.csr_dst, 30)
        assert np.all(d[2:] <= 0.85 * d[1:-1] * (1 + 1e-9) + 1e-18)
        assert d[1] > 0


def test_pr_deltas_cycle_is_stationary():
    g = directed_cycle(64)
    d = oracle.pagerank_deltas(g.n, g.csr_off, g.csr_dst, 5)
    assert np.all(d <= 64 * 2.0 ** -52 / 64)


def test_pr_converge_equals_fixed_run():
    g = random_graph(400, 2400, seed=7)
    res, T, d = oracle.pagerank_converge(g, 1e-6, 200)
    assert 1 <= T < 200 and d[T] < 1e-6 and np.all(d[1:T] >= 1e-6)
    fixed = oracle.run_graph("pagerank", g, T)
    assert np.array_equal(res.values, fixed.values)
    assert res.supersteps == T + 1
    # never below the tolerance: runs the cap
    _, T2, _ = oracle.pagerank_converge(g, 0.0, 15)
    assert T2 == 15


# ------------------------------------------------ PageRank, general damping --

def _dense_pr(g, T, d):
    # r <- (1-d)/N + d * A^T (D^+ r): the matrix form of Fig. 8 with damping d
    # (Ligra's Fig. 16 form), dense numpy, dangling mass dropped.
    A = adjacency(g).toarray()
    outdeg = A.sum(axis=1)
    dinv = np.where(outdeg > 0, 1.0 / np.where(outdeg > 0, outdeg, 1), 0.0)
    r = np.full(g.n, 1.0 / g.n)
    for _ in range(T):
        r = (1.0 - d) / g.n + d * (A.T @ (dinv * r))
    return r


@pytest.mark.parametrize("d", [0.3, 0.6, 0.99, 1.0])
@pytest.mark.parametrize("seed", [1, 2])
def test_pr_general_damping_matches_matrix_form(d, seed):
    g = random_graph(120, 700, seed=seed, loops=True, dups=True)
    for T in (1, 4, 10):
        r = oracle.run_graph("pagerank", g, T, damping=d)
        assert r.status == oracle.OK
        np.testing.assert_allclose(r.values, _dense_pr(g, T, d), rtol=1e-13, atol=0)


def test_pr_damping_half_exact_rationals():
    # d = 1/2: the exact rational iterate r <- 1/(2N) + 1/2 * sum of the
    # in-neighbours' r/outdeg, on a multigraph with self-loops and a dangling
    # vertex; the double result is within 1e-14 relative of it.
    n = 9
    src = [0, 0, 1, 2, 2, 3, 4, 4, 5, 6, 6, 7, 1, 3]
    dst = [1, 1, 2, 0, 3, 3, 5, 0, 6, 7, 2, 4, 4, 8]
    g = graphgen.from_edges(n, src, dst, keep_self_loops=True, keep_duplicates=True)
    half = Fraction(1, 2)
    r = [Fraction(1, n)] * n
    for T in range(1, 8):
        acc = [Fraction(0)] * n
        for u, v in zip(src, dst):
            acc[v] += r[u] / src.count(u)
        r = [(1 - half) / n + half * a for a in acc]
        got = oracle.run_graph("pagerank", g, T, damping=0.5).values
        exact = np.array([float(x) for x in r])
        np.testing.assert_allclose(got, exact, rtol=1e-14, atol=0)


@pytest.mark.parametrize("d", [0.2, 0.7])
def test_pr_general_damping_mass_balance(d):
    # sum r_{k+1} = (1-d) + d * (sum r_k - sum of the dangling r_k)
    g = random_graph(400, 1500, seed=9)
    dangling = np.diff(g.csr_off) == 0
    assert dangling.any()
    prev = oracle.run_graph("pagerank", g, 0, damping=d).values
    for T in range(1, 8):
        cur = oracle.run_graph("pagerank", g, T, damping=d).values
        expect = (1.0 - d) + d * (prev.sum() - prev[dangling].sum())
        assert abs(cur.sum() - expect) <= 1e-13
        prev = cur


@pytest.mark.parametrize("d", [0.0, -0.5, 1.5, float("nan")])
def test_pr_damping_out_of_range_rejected(d):
    g = directed_cycle(5)
    assert oracle.run_graph("pagerank", g, 3, damping=d).status == oracle.EINVAL
    assert oracle.run_pull("pagerank", g, 3, damping=d).status == oracle.EINVAL
