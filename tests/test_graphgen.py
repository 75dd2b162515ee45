"""Input generators: determinism, structure and the recipe's invariants."""
import numpy as np
import pytest

import graphgen
from tests.graphs_small import edge_arrays


def _edge_set(g):
    s, d = edge_arrays(g)
    return set(zip(s.tolist(), d.tolist()))


def test_rmat_deterministic_and_clean():
    a = graphgen.rmat(12, 16, seed=7)
    b = graphgen.rmat(12, 16, seed=7)
    c = graphgen.rmat(12, 16, seed=8)
    assert np.array_equal(a.csr_off, b.csr_off) and np.array_equal(a.csr_dst, b.csr_dst)
    assert not np.array_equal(a.csr_dst[:1000], c.csr_dst[:1000])
    s, d = edge_arrays(a)
    assert not (s == d).any()                        # no self-loops
    key = s * a.n + d
    assert np.all(np.diff(key) > 0)                  # sorted and duplicate-free
    assert a.csr_off[0] == 0 and a.csr_off[-1] == a.csr_dst.size


def test_rmat_skew_hub_at_zero():
    # Unpermuted R-MAT with a = 0.57 concentrates edges on low ids.
    g = graphgen.rmat(14, 16, seed=1)
    od = np.diff(g.csr_off)
    assert od[0] == od.max()
    assert g.m > 0.8 * 16 * g.n


def test_csc_is_transpose():
    g = graphgen.rmat(11, 8, seed=3)
    s, d = edge_arrays(g)
    ts = np.repeat(np.arange(g.n), np.diff(g.csc_off).astype(np.int64))
    assert set(zip(d.tolist(), s.tolist())) == set(zip(ts.tolist(), g.csc_src.tolist()))
    for v in range(0, g.n, 97):
        lst = g.csc_src[g.csc_off[v]:g.csc_off[v + 1]]
        assert np.all(np.diff(lst) > 0)


def test_symmetrised_is_symmetric():
    g = graphgen.rmat(11, 16, seed=2, symmetric=True)
    e = _edge_set(g)
    assert all((v, u) in e for (u, v) in e)
    assert g.csc_src is g.csr_dst


def test_weights_symmetric_and_in_range():
    g = graphgen.grid_with_shortcuts(32, 0.01, seed=3)
    assert g.csr_w.min() >= 1 and g.csr_w.max() <= 255
    s, d = edge_arrays(g)
    w = {(u, v): x for u, v, x in zip(s.tolist(), d.tolist(), g.csr_w.tolist())}
    assert all(w[(v, u)] == x for (u, v), x in w.items())
    grid_edges = 2 * 32 * 31
    assert g.meta["shortcuts"] == int(0.01 * grid_edges)
    assert g.m == 2 * (grid_edges + g.meta["shortcuts"])


def test_duplicates_and_loops_kept_on_request():
    g = graphgen.from_edges(3, [0, 0, 1, 2], [1, 1, 1, 0], keep_self_loops=True, keep_duplicates=True)
    assert g.csr_dst.tolist() == [1, 1, 1, 0]
    g = graphgen.from_edges(3, [0, 0, 1, 2], [1, 1, 1, 0])
    assert g.csr_dst.tolist() == [1, 0]


def test_small_family_sizes():
    fam = graphgen.small_graph_family(count=6, seed=41)
    for g in fam:
        assert 2 ** 10 <= g.n <= 2 ** 16
        assert g.csr_off[-1] == g.csr_dst.size


def test_pick_sources_distinct_and_eligible():
    g = graphgen.rmat(12, 16, seed=4, symmetric=True)
    src = graphgen.pick_sources(g, 64, seed=40)
    assert len(set(src.tolist())) == 64
    assert (np.diff(g.csr_off)[src] > 0).all()


def test_disjoint_union_renumbers_and_records_parts():
    from tests.graphs_small import edge_arrays, random_graph

    gs = [random_graph(10, 30, seed=1), random_graph(7, 12, seed=2), random_graph(5, 0, seed=3)]
    u = graphgen.disjoint_union(gs)
    assert u.n == 22 and u.m == sum(g.m for g in gs)
    assert u.meta["parts"].tolist() == [0, 10, 17, 22]
    us, ud = edge_arrays(u)
    base = 0
    want_s, want_d = [], []
    for g in gs:
        s, d = edge_arrays(g)
        want_s += list(s + base)
        want_d += list(d + base)
        base += g.n
    assert us.tolist() == want_s and ud.tolist() == want_d
    # CSC of the union is the union of the CSCs
    cs = np.repeat(np.arange(u.n), np.diff(u.csc_off).astype(np.int64))
    assert sorted(zip(u.csc_src.tolist(), cs.tolist())) == sorted(zip(us.tolist(), ud.tolist()))


@pytest.mark.parametrize("scale,seed", [(10, 5), (14, 5), (16, 2)])
def test_symmetrise_equals_symmetric_draw(scale, seed):
    # merging the directed CSR and CSC gives the graph a symmetric draw of the
    # same edge list builds (reverses added, loops and duplicates dropped)
    d = graphgen.rmat(scale, 16, seed=seed)
    s = graphgen.rmat(scale, 16, seed=seed, symmetric=True)
    m = graphgen.symmetrise(d)
    assert m.symmetric and m.csc_src is m.csr_dst
    assert np.array_equal(m.csr_off, s.csr_off)
    assert np.array_equal(m.csr_dst, s.csr_dst)
    assert m.name == s.name


def test_symmetrise_small_cases():
    e = graphgen.symmetrise(graphgen.from_edges(4, [], []))
    assert e.m == 0 and np.array_equal(e.csr_off, np.zeros(5, np.uint64))
    g = graphgen.from_edges(3, [0, 1, 2, 2], [1, 0, 2, 0], keep_self_loops=True)
    m = graphgen.symmetrise(g)
    assert m.csr_off.tolist() == [0, 2, 3, 4]
    assert m.csr_dst.tolist() == [1, 2, 0, 0]
