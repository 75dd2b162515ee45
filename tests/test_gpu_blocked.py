"""GPU parity of PageRank's blocked pull (graph flag IPG_GRAPH_BLOCKED) against
the CPU oracle, through the C ABI.

The blocked pull adds the same messages under the sum combiner of Fig. 8, but
in an order that varies from run to run (LDS atomics), so -- as for push --
ranks are compared with the oracle within the PageRank tolerance (max
relative error <= 1e-12), at every update where the case is small.  Cases
span: one destination block with one slice and with many slices (partial
sums + the finish launch), many blocks, sources beyond the first window of
65536, the plain and the hot-first store, blocks and rows without in-edges,
the usual edge cases, disjoint unions, convergence runs, graph replay and the
full-size symmetrised R-MAT scale 20 graph.
"""
import numpy as np
import pytest

import graphgen
import oracle
from tests.graphs_small import random_graph

pytestmark = pytest.mark.gpu

PR_RTOL = 1e-12
OFF = 0xFFFFFFFF


@pytest.fixture(scope="module")
def ipg():
    import torch

    import paper_2010_08781_amd as m

    assert torch.cuda.is_available()
    m.lib()
    return m


def max_rel(a, b):
    return float(np.max(np.abs(a - b) / np.abs(b))) if b.size else 0.0


def check(ipg, hg, Ts, rename=True, modes=("pull",)):
    g = ipg.Graph.from_host(hg, rename=rename, blocked=True)
    for T in Ts:
        ref = oracle.run_graph("pagerank", hg, T)
        for mode in modes:
            vals, st = g.run("pagerank", T, mode=mode)
            err = max_rel(ipg.values_to_numpy(vals), ref.values)
            assert err <= PR_RTOL, f"T={T} {mode} rename={rename}: max rel err {err:.3e}"
            assert st.supersteps == T + 1 and np.array_equal(st.trace, ref.trace)
    return g


@pytest.mark.parametrize("rename", [True, False])
def test_one_block_many_slices_every_update(ipg, rename):
    # N = 16384 < one block of 20224 rows; E = 262K edges -> 4 slices whose
    # partial sums the finish launch adds.
    hg = graphgen.workload("rmat-s14-dir")
    check(ipg, hg, Ts=tuple(range(0, 11)), rename=rename)


@pytest.mark.parametrize("sym", [False, True])
def test_many_blocks_and_windows(ipg, sym):
    # N = 131072: 7 blocks (the last one partial) and two source windows.
    hg = graphgen.rmat(17, 16, seed=21, symmetric=sym)
    check(ipg, hg, Ts=(1, 2, 10), rename=True)
    check(ipg, hg, Ts=(3,), rename=False)


def test_one_slice_blocks_and_empty_blocks(ipg):
    # Few edges per block (every block one slice, finished by its own
    # workgroup) and a range of high ids without in-edges: whole blocks with
    # no edges still produce 0.15/N.
    n = 90000
    rng = np.random.default_rng(6)
    src = rng.integers(0, n, 30000)
    dst = rng.integers(0, 40000, 30000)
    hg = graphgen.from_edges(n, src, dst)
    check(ipg, hg, Ts=(0, 1, 2, 10), rename=False)
    check(ipg, hg, Ts=(10,), rename=True)


def test_hub_rows_and_ragged_chunks(ipg):
    # A destination with in-degree far above a chunk, a source with a huge
    # out-degree (one source feeding many chunks), and N not a multiple of 64.
    n = 5000
    rng = np.random.default_rng(4)
    src = np.concatenate([np.arange(1, n), rng.integers(0, n, 20000), np.zeros(3000, np.int64)])
    dst = np.concatenate([np.zeros(n - 1, np.int64), rng.integers(0, n, 20000), rng.integers(1, n, 3000)])
    hg = graphgen.from_edges(n, src, dst)
    check(ipg, hg, Ts=(1, 2, 10), modes=("pull", "push"))


@pytest.mark.parametrize("case", ["loops_dups", "single", "no_edges", "cycle", "dense"])
def test_edge_cases(ipg, case):
    if case == "loops_dups":
        hg = random_graph(333, 3000, seed=3, loops=True, dups=True)
    elif case == "single":
        hg = graphgen.from_edges(1, [], [])
    elif case == "no_edges":
        hg = graphgen.from_edges(70, [], [])
    elif case == "cycle":
        n = 1000
        hg = graphgen.from_edges(n, np.arange(n), (np.arange(n) + 1) % n)
    else:  # few vertices, many edges: many slices of one small block
        hg = random_graph(300, 400000, seed=9, loops=True, dups=True)
    check(ipg, hg, Ts=(0, 1, 5, 10))


def test_item_kernels_when_switched_off(ipg):
    # tuning blocked = UINT32_MAX runs the row-item pull, bitwise equal to
    # the same store without blocked in-edges
    import torch

    hg = graphgen.rmat(15, 16, seed=8, symmetric=True)
    a = ipg.Graph.from_host(hg, blocked=True)
    b = ipg.Graph.from_host(hg, blocked=False)
    ra, _ = a.run("pagerank", 10, mode="pull", tuning={"blocked": OFF})
    rb, _ = b.run("pagerank", 10, mode="pull")
    assert torch.equal(ra, rb)
    rc, _ = a.run("pagerank", 10, mode="pull")
    assert max_rel(ipg.values_to_numpy(rc), ipg.values_to_numpy(rb)) <= PR_RTOL


def test_parts_converge_and_replay(ipg):
    import torch

    graphs = [graphgen.rmat_small(n, 8, seed=700 + n) for n in (1500, 30000, 900, 22000)]
    u = graphgen.disjoint_union(graphs)
    g = ipg.Graph.from_host(u, blocked=True)
    parts = torch.from_numpy(u.meta["parts"].astype(np.int32)).cuda()
    # each part's ranks equal a separate run on that part
    r, _ = g.run("pagerank", 10, parts=parts)
    r = ipg.values_to_numpy(r)
    off = u.meta["parts"]
    for i, hg in enumerate(graphs):
        ref = oracle.run_graph("pagerank", hg, 10)
        assert max_rel(r[off[i]:off[i + 1]], ref.values) <= PR_RTOL, i
    # to convergence: the stopping update is the oracle's (tolerance placed
    # away from every change of the run)
    hg = graphs[1]
    gb = ipg.Graph.from_host(hg, blocked=True)
    d = oracle.pagerank_deltas(hg.n, hg.csr_off, hg.csr_dst, 200)
    tol = 1e-9
    while np.any(np.abs(d[1:] - tol) <= max(1e-6 * tol, 1e-12)):
        tol *= 1.37
    ref, T, _ = oracle.pagerank_converge(hg, tol, 200)
    c, st = gb.run("pagerank", 200, mode="pull", tol=tol)
    assert st.supersteps == T + 1 and max_rel(ipg.values_to_numpy(c), ref.values) <= PR_RTOL
    np.testing.assert_allclose(st.residual[1:], d[1:T + 1], rtol=1e-9, atol=1e-13)
    # graph replay, several times with eager work in between
    ref = oracle.run_graph("pagerank", hg, 10)
    for _ in range(3):
        rr, _ = gb.run("pagerank", 10, mode="pull", graph=True)
        assert max_rel(ipg.values_to_numpy(rr), ref.values) <= PR_RTOL
        e, _ = gb.run("pagerank", 4, mode="pull")
        assert max_rel(ipg.values_to_numpy(e), oracle.run_graph("pagerank", hg, 4).values) <= PR_RTOL


def test_more_row_blocks_than_slices(ipg):
    # 8.4M vertices: 415 row-capped blocks, more than the 256 slices of a
    # wave, so blocks run in rounds; dense rows form narrow blocks and the
    # costliest are cut into slices with partial sums
    hg = graphgen.rmat(23, 4, seed=5)
    g = ipg.Graph.from_host(hg, blocked=True)
    for T in (1, 3):
        ref = oracle.run_graph("pagerank", hg, T)
        vals, st = g.run("pagerank", T, mode="pull")
        assert max_rel(ipg.values_to_numpy(vals), ref.values) <= PR_RTOL
        assert np.array_equal(st.trace, ref.trace)
    ref = oracle.run_graph("cc", hg, 0)
    for persistent in (False, True):
        vals, st = g.run("cc", mode="pull", persistent=persistent)
        assert np.array_equal(ipg.values_to_numpy(vals), ref.values) and np.array_equal(st.trace, ref.trace)
    # unit-weight SSSP with both exchanges: in the device-driven loop the
    # compute's grid (over 8.4M vertices) is capped to the push grid in the
    # shared launch, and push supersteps queue pieces
    ref = oracle.run_graph("sssp", hg, 0, source=0, weighted=False)
    for mode in ("auto", "push"):
        for persistent in (False, True):
            vals, st = g.run("sssp", source=0, mode=mode, persistent=persistent)
            assert np.array_equal(ipg.values_to_numpy(vals), ref.values), (mode, persistent)
            assert np.array_equal(st.trace, ref.trace), (mode, persistent)


def test_full_size_rmat_s20_symmetrised(ipg):
    # the benchmark's graph and launch path (hot-first store + blocked in-edges)
    hg = graphgen.workload("rmat-s20-sym")
    g = ipg.Graph.from_host(hg, blocked=True)
    ref = oracle.run_graph("pagerank", hg, 10)
    vals, st = g.run("pagerank", 10, mode="pull")
    assert max_rel(ipg.values_to_numpy(vals), ref.values) <= PR_RTOL
    vals, st = g.run("pagerank", 10, mode="pull", graph=True)
    assert max_rel(ipg.values_to_numpy(vals), ref.values) <= PR_RTOL


# ---------------------------------------------------------------- CC / SSSP --
# The blocked min-pull combines with atomic minima, which do not depend on
# the order: values and per-superstep traces are bit-exact.

def check_min(ipg, hg, app, source=0, rename=True, weighted=True, modes=("pull", "auto", "push")):
    ref = oracle.run_graph(app, hg, 0, source=source, weighted=weighted)
    assert ref.status == oracle.OK
    g = ipg.Graph.from_host(hg, weighted=weighted, rename=rename, blocked=True)
    for mode in modes:
        for persistent in (False, True):
            vals, st = g.run(app, source=source, mode=mode, persistent=persistent)
            got = ipg.values_to_numpy(vals)
            assert np.array_equal(got, ref.values), f"{app} {mode} persistent={persistent}: {np.sum(got != ref.values)} differ"
            assert np.array_equal(st.trace, ref.trace), (app, mode, persistent)
            assert st.halted
    return g


@pytest.mark.parametrize("rename", [True, False])
@pytest.mark.parametrize("app", ["cc", "sssp"])
def test_min_pull_rmat_s16_symmetrised(ipg, app, rename):
    check_min(ipg, graphgen.rmat(16, 16, seed=31, symmetric=True), app, source=3, rename=rename)


@pytest.mark.parametrize("app", ["cc", "sssp"])
def test_min_pull_directed_and_multigraph(ipg, app):
    check_min(ipg, graphgen.workload("rmat-s14-dir"), app, source=0)
    check_min(ipg, random_graph(3000, 40000, seed=5, loops=True, dups=True), app, source=17, rename=False)


def test_min_pull_long_path_and_edge_cases(ipg):
    from tests.graphs_small import path
    check_min(ipg, path(3000), "sssp", source=0, modes=("pull", "auto"))
    check_min(ipg, path(3000), "cc", modes=("pull",))
    for hg in (graphgen.from_edges(1, [], []), graphgen.from_edges(70, [], []),
               graphgen.from_edges(90000, np.arange(0, 300), np.arange(1, 301))):
        for app in ("cc", "sssp"):
            check_min(ipg, hg, app, source=0, modes=("pull", "auto"))


def test_min_pull_weighted_sssp_uses_row_items(ipg):
    # weighted SSSP keeps the row-item pull on a blocked store; still exact
    check_min(ipg, graphgen.grid_with_shortcuts(256, 0.02, seed=7), "sssp", source=0, modes=("pull", "auto"))


def test_min_pull_full_size_and_switched_off(ipg):
    import torch

    hg = graphgen.workload("rmat-s20-sym")
    g = check_min(ipg, hg, "cc", modes=("pull", "auto"))
    for app in ("cc", "sssp"):
        a, sa = g.run(app, mode="pull", persistent=True)
        b, sb = g.run(app, mode="pull", persistent=True, tuning={"blocked": OFF})
        assert torch.equal(a, b) and np.array_equal(sa.trace, sb.trace)
    ref = oracle.run_graph("sssp", hg, 0, source=0)
    v, st = g.run("sssp", source=0, mode="auto", persistent=True)
    assert np.array_equal(ipg.values_to_numpy(v), ref.values) and np.array_equal(st.trace, ref.trace)


# ------------------------------------------------- binned cold sources ----

def check_binned(ipg, hg, Ts, hot=65536, rename=True, modes=("pull",), min_apps=True):
    g = ipg.Graph.from_host(hg, rename=rename, blocked=True, binned=True, binned_hot=hot)
    for T in Ts:
        ref = oracle.run_graph("pagerank", hg, T)
        for mode in modes:
            print(f"[binned] {hg.name} T={T} {mode} rename={rename} hot={hot}", flush=True)
            vals, st = g.run("pagerank", T, mode=mode)
            err = max_rel(ipg.values_to_numpy(vals), ref.values)
            assert err <= PR_RTOL, f"T={T} {mode}: max rel err {err:.3e}"
            assert st.supersteps == T + 1 and np.array_equal(st.trace, ref.trace)
    if min_apps:
        # CC and SSSP over the binned in-edges of the caller's ids: every
        # exchange, both loops, the sender gate on (default) and off
        for app in ("cc", "sssp"):
            ref = oracle.run_graph(app, hg, 0, weighted=False)
            for mode in ("pull", "auto"):
                for persistent in (False, True):
                    for tuning in (None, {"gate_div": 0xFFFFFFFF}, {"gate_div": 1}):
                        print(f"[binned] {hg.name} {app} {mode} persistent={persistent} tuning={tuning}", flush=True)
                        vals, st = g.run(app, source=0, mode=mode, persistent=persistent, tuning=tuning)
                        assert np.array_equal(ipg.values_to_numpy(vals), ref.values), (app, mode, persistent, tuning)
                        assert np.array_equal(st.trace, ref.trace), (app, mode, persistent, tuning)
    return g


@pytest.mark.parametrize("rename", [True, False])
def test_binned_rmat_s17_every_update(ipg, rename):
    # N = 131072: sources from 65536 on binned, the rest gathered
    check_binned(ipg, graphgen.rmat(17, 16, seed=21), Ts=tuple(range(0, 11)), rename=rename)


def test_binned_symmetrised_and_switched_off(ipg):
    hg = graphgen.rmat(18, 16, seed=4, symmetric=True)
    g = check_binned(ipg, hg, Ts=(1, 10))
    ref = oracle.run_graph("pagerank", hg, 10)
    vals, _ = g.run("pagerank", 10, mode="pull", tuning={"blocked": 0xFFFFFFFF})  # row items on the same store
    assert max_rel(ipg.values_to_numpy(vals), ref.values) <= PR_RTOL
    # CC and SSSP on the symmetric binned store run under the hot-first names
    # on PageRank's table; with the blocked pull switched off, on the caller's
    # names with row items
    for app in ("cc", "sssp"):
        r = oracle.run_graph(app, hg, 0)
        for persistent in (False, True):
            for tuning in (None, {"blocked": 0xFFFFFFFF}):
                v, st = g.run(app, source=0, persistent=persistent, tuning=tuning)
                assert np.array_equal(ipg.values_to_numpy(v), r.values) and np.array_equal(st.trace, r.trace)


@pytest.mark.parametrize("app", ["cc", "sssp"])
def test_symmetric_binned_runs_under_new_names(ipg, app):
    # Sources mapped to their new names, CC labels started from the caller's
    # ids, values mapped back: every exchange, both loops, several sources,
    # and a graph with isolated vertices and several components (the labels
    # are the smallest caller id of each component, not of its new names).
    n = 70000
    rng = np.random.default_rng(31)
    a = rng.integers(0, 40000, 300000)
    b = np.minimum(a + rng.integers(1, 3000, 300000), 39999)  # one component among 0..39999, mostly
    c = rng.integers(45000, 60000, 50000)
    d = rng.integers(45000, 60000, 50000)                       # another among 45000..59999; the rest isolated
    hg = graphgen.from_edges(n, np.concatenate([a, c]), np.concatenate([b, d]), symmetric=True)
    g = ipg.Graph.from_host(hg, blocked=True, binned=True, binned_hot=4096)
    sources = [0] if app == "cc" else [0, 45000, 65000, int(graphgen.pick_sources(hg, 1, seed=3)[0])]
    for src in sources:
        ref = oracle.run_graph(app, hg, 0, source=src)
        for mode in ("auto", "push", "pull"):
            for persistent in (False, True):
                print(f"[renamed] {app} src={src} {mode} persistent={persistent}", flush=True)
                v, st = g.run(app, source=src, mode=mode, persistent=persistent)
                assert np.array_equal(ipg.values_to_numpy(v), ref.values), (src, mode, persistent)
                assert np.array_equal(st.trace, ref.trace), (src, mode, persistent)


def test_symmetric_binned_weighted_sssp_keeps_caller_names(ipg):
    # weighted SSSP on a symmetric binned store: the renamed CSC has no weights,
    # so the run keeps the caller's names (row-item pull with CSC weights)
    hg = graphgen.grid_with_shortcuts(128, 0.01, seed=5)
    assert hg.csr_w is not None
    g = ipg.Graph.from_host(hg, blocked=True, binned=True, binned_hot=1024)
    ref = oracle.run_graph("sssp", hg, 0, source=7)
    for mode in ("auto", "pull", "push"):
        for persistent in (False, True):
            v, st = g.run("sssp", source=7, mode=mode, persistent=persistent)
            assert np.array_equal(ipg.values_to_numpy(v), ref.values) and np.array_equal(st.trace, ref.trace)


def test_binned_multigraph_hubs_and_empty_ranges(ipg):
    n = 300000
    rng = np.random.default_rng(8)
    src = np.concatenate([rng.integers(0, n, 400000), np.full(50000, 250001), rng.integers(0, n, 30000)])
    dst = np.concatenate([rng.integers(0, 200000, 400000), rng.integers(0, 200000, 50000), np.zeros(30000, np.int64)])
    hg = graphgen.from_edges(n, src, dst, keep_self_loops=True, keep_duplicates=True)
    check_binned(ipg, hg, Ts=(0, 1, 3, 10), rename=False)
    check_binned(ipg, hg, Ts=(10,), rename=True, hot=1)


def test_binned_cold_only_and_convergence(ipg):
    # every edge from one cold window; a convergence run and a replayed graph on the binned store
    n = 140000
    rng = np.random.default_rng(2)
    hg = graphgen.from_edges(n, rng.integers(131072, 131072 + 16384, 60000), rng.integers(0, n, 60000))
    g = check_binned(ipg, hg, Ts=(1, 2, 10), rename=False)
    want, T, _ = oracle.pagerank_converge(hg, 1e-9, 60)
    vals, st = g.run("pagerank", 60, mode="pull", tol=1e-9)
    assert st.supersteps == T + 1 and max_rel(ipg.values_to_numpy(vals), want.values) <= PR_RTOL
    ref = oracle.run_graph("pagerank", hg, 10)
    for _ in range(3):
        vals, _ = g.run("pagerank", 10, mode="pull", graph=True)
        assert max_rel(ipg.values_to_numpy(vals), ref.values) <= PR_RTOL
