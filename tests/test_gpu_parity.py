"""GPU parity: the HIP superstep engine against the CPU oracle, through the C ABI.

CC and SSSP: values and the per-superstep trace (active, senders, messages)
bit-exact.  PageRank (FP64): max relative error <= 1e-12 at every superstep
(checked by running T = 1..10 updates; the T-th iterate does not depend on
how many updates follow).  The exchange mode (push / pull / auto) never
changes results.
"""
import numpy as np
import pytest

import graphgen
import oracle
from tests.graphs_small import path, random_graph

pytestmark = pytest.mark.gpu

PR_RTOL = 1e-12


@pytest.fixture(scope="module")
def ipg():
    import torch

    import paper_2010_08781_amd as m

    assert torch.cuda.is_available()
    m.lib()
    return m


def to_np(t):
    import paper_2010_08781_amd as m

    return m.values_to_numpy(t)


def max_rel(a, b):
    return float(np.max(np.abs(a - b) / np.abs(b))) if b.size else 0.0


def check_min_app(ipg, hg, app, source=0, modes=("push", "pull", "auto"), weighted=True):
    ref = oracle.run_graph(app, hg, 0, source=source, weighted=weighted)
    assert ref.status == oracle.OK
    g = ipg.Graph.from_host(hg, weighted=weighted)
    for mode in modes:
        vals, st = g.run(app, source=source, mode=mode)
        got = to_np(vals)
        assert np.array_equal(got, ref.values), f"{app} {mode}: {np.sum(got != ref.values)} values differ"
        assert st.supersteps == ref.supersteps, (mode, st.supersteps, ref.supersteps)
        assert np.array_equal(st.trace, ref.trace), f"{app} {mode} trace\n{st.trace}\n{ref.trace}"
        assert st.halted
    return g


def check_pagerank(ipg, hg, Ts=(0, 1, 2, 3, 10), modes=("pull", "push")):
    g = ipg.Graph.from_host(hg)
    for T in Ts:
        ref = oracle.run_graph("pagerank", hg, T)
        for mode in modes:
            vals, st = g.run("pagerank", T, mode=mode)
            got = to_np(vals)
            err = max_rel(got, ref.values)
            assert err <= PR_RTOL, f"T={T} {mode}: max rel err {err:.3e}"
            assert st.supersteps == T + 1
            assert np.array_equal(st.trace, ref.trace)
    return g


# ------------------------------------------------------------ PageRank ----

def test_pagerank_rmat_s14_every_superstep(ipg):
    # R-MAT scale 14, edge factor 16, directed, seed 1; T = 1..10.
    hg = graphgen.workload("rmat-s14-dir")
    check_pagerank(ipg, hg, Ts=tuple(range(0, 11)))


@pytest.mark.parametrize("d", [0.5, 0.6, 0.99])
def test_pagerank_damping(ipg, d):
    # damping d != 0.85 (rank = (1-d)/N + d * sum) in every exchange and store:
    # row items, blocked in-edges, push, the replayed graph, and a
    # convergence run; trace counted on the device
    hg = graphgen.workload("rmat-s14-dir")
    plain = ipg.Graph.from_host(hg, rename=False)
    blocked = ipg.Graph.from_host(hg, blocked=True)
    for T in (1, 4, 10):
        ref = oracle.run_graph("pagerank", hg, T, damping=d)
        for g, mode, graph in ((plain, "pull", False), (plain, "push", False), (blocked, "pull", False),
                               (blocked, "pull", True)):
            vals, st = g.run("pagerank", T, mode=mode, damping=d, graph=graph)
            err = max_rel(to_np(vals), ref.values)
            assert err <= PR_RTOL, f"d={d} T={T} {mode} graph={graph}: {err:.3e}"
            assert np.array_equal(st.trace, ref.trace)
    want, T, _ = oracle.pagerank_converge(hg, 1e-6, 100, damping=d)
    vals, st = blocked.run("pagerank", 100, mode="pull", damping=d, tol=1e-6)
    assert st.supersteps == T + 1
    assert max_rel(to_np(vals), want.values) <= PR_RTOL
    assert np.array_equal(st.trace, want.trace)


def test_pagerank_damping_rejected(ipg):
    g = ipg.Graph.from_host(graphgen.workload("rmat-s14-dir"))
    for d in (-0.1, 1.5, float("nan")):
        with pytest.raises(ipg.IpgError):
            g.run("pagerank", 3, damping=d)


def test_pagerank_pull_bitwise_deterministic(ipg):
    hg = graphgen.workload("rmat-s14-dir")
    g = ipg.Graph.from_host(hg)
    a = to_np(g.run("pagerank", 10, mode="pull")[0])
    b = to_np(g.run("pagerank", 10, mode="pull")[0])
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))


def test_pagerank_superstep_times(ipg):
    # per-superstep times from the timing events between the launches: one
    # per superstep, each positive, together within the run's time (the run
    # also maps the ranks back after the last superstep); the ranks are the
    # those of a run without per-superstep timing
    hg = graphgen.workload("rmat-s14-dir")
    g = ipg.Graph.from_host(hg, blocked=True)
    for _ in range(3):
        vals, st = g.run("pagerank", 10, mode="pull", timing=True)
        assert st.usec.shape == (11,) and (st.usec > 0).all()
        assert st.seconds > 0 and st.usec.sum() <= st.seconds * 1e6 * 1.001 + 1.0
        plain, st2 = g.run("pagerank", 10, mode="pull", timing=False)
        assert st2.seconds > 0
        assert max_rel(to_np(vals), to_np(plain)) <= PR_RTOL  # blocked sums: order may vary


def test_pagerank_long_rows_and_hubs(ipg):
    # A hub with in-degree far above the LDS tile (long-row path) plus a
    # ragged tail of small rows; N not a multiple of 64.
    n = 5000
    rng = np.random.default_rng(4)
    src = np.concatenate([np.arange(1, n), rng.integers(0, n, 20000), np.zeros(3000, np.int64)])
    dst = np.concatenate([np.zeros(n - 1, np.int64), rng.integers(0, n, 20000), rng.integers(1, n, 3000)])
    hg = graphgen.from_edges(n, src, dst)
    assert np.diff(hg.csc_off).max() > 2048
    check_pagerank(ipg, hg, Ts=(1, 2, 10))


@pytest.mark.parametrize("case", ["loops_dups", "single", "no_edges", "cycle"])
def test_pagerank_edge_cases(ipg, case):
    if case == "loops_dups":
        hg = random_graph(333, 3000, seed=3, loops=True, dups=True)
    elif case == "single":
        hg = graphgen.from_edges(1, [], [])
    elif case == "no_edges":
        hg = graphgen.from_edges(70, [], [])
    else:
        n = 1000
        hg = graphgen.from_edges(n, np.arange(n), (np.arange(n) + 1) % n)
    check_pagerank(ipg, hg, Ts=(0, 1, 5, 10))


# ------------------------------------------------------------------ CC ----

def test_cc_rmat_s20_symmetrised(ipg):
    # Symmetrised R-MAT scale 20, edge factor 16, seed 2 (the CC/SSSP workload).
    hg = graphgen.workload("rmat-s20-sym")
    check_min_app(ipg, hg, "cc")


@pytest.mark.parametrize("sym", [True, False])
def test_cc_random_and_directed(ipg, sym):
    hg = random_graph(20000, 30000, seed=8, symmetric=sym)
    check_min_app(ipg, hg, "cc")


@pytest.mark.parametrize("case", ["path", "no_edges", "single", "loops_dups", "hub"])
def test_cc_edge_cases(ipg, case):
    if case == "path":
        hg = path(300)
    elif case == "no_edges":
        hg = graphgen.from_edges(130, [], [])
    elif case == "single":
        hg = graphgen.from_edges(1, [0], [0], keep_self_loops=True)
    elif case == "loops_dups":
        hg = random_graph(500, 1500, seed=6, loops=True, dups=True)
    else:
        n = 9000
        hg = graphgen.from_edges(n, np.full(n - 1, n - 1), np.arange(n - 1), symmetric=True)
    check_min_app(ipg, hg, "cc")


# ---------------------------------------------------------------- SSSP ----

def test_sssp_rmat_s20_symmetrised_from_0(ipg):
    hg = graphgen.workload("rmat-s20-sym")
    check_min_app(ipg, hg, "sssp", source=0)


@pytest.mark.parametrize("source", [0, 77])
def test_sssp_directed_random(ipg, source):
    hg = random_graph(20000, 60000, seed=9)
    check_min_app(ipg, hg, "sssp", source=source)


def test_sssp_weighted_grid(ipg):
    hg = graphgen.grid_with_shortcuts(256, 0.01, seed=3)
    check_min_app(ipg, hg, "sssp", source=0)
    check_min_app(ipg, hg, "sssp", source=0, weighted=False, modes=("auto",))


def test_sssp_weighted_directed_with_loops(ipg):
    hg = random_graph(3000, 20000, seed=10, loops=True, dups=True, weight_seed=3)
    check_min_app(ipg, hg, "sssp", source=5)


def test_push_frontier_list_dense_transitions(ipg):
    # SSSP from a hub on a symmetrised R-MAT: the push frontier goes from a
    # short list (the source) to a dense sweep of the mailboxes and back to
    # a list; every transition must keep values and traces exact.
    hg = graphgen.rmat(16, 16, seed=6, symmetric=True)
    ref = oracle.run_graph("sssp", hg, 0, source=0)
    g = ipg.Graph.from_host(hg)
    vals, st = g.run("sssp", source=0, mode="push")
    assert np.array_equal(to_np(vals), ref.values)
    assert np.array_equal(st.trace, ref.trace)
    limit = max(4096, hg.n // 16)
    sizes = ref.trace[1:, 0]
    assert (sizes > limit).any() and (sizes[sizes > 0] <= limit).any()


# ------------------------------------------------------------ boundary ----

def test_cap_returns_not_converged(ipg):
    hg = path(50)
    g = ipg.Graph.from_host(hg)
    ref = oracle.run_graph("cc", hg, 7)
    assert ref.status == oracle.NOT_CONVERGED
    vals, st = g.run("cc", 7)
    assert st.status == ipg.NOT_CONVERGED and st.supersteps == 7
    assert np.array_equal(to_np(vals), ref.values)


def test_errors(ipg):
    import torch

    hg = random_graph(100, 300, seed=1)
    g = ipg.Graph.from_host(hg)
    with pytest.raises(ipg.IpgError) as e:
        g.run("cc", combiner=ipg.COMBINE_SUM)
    assert e.value.status == ipg.EUNSUPPORTED
    with pytest.raises(ipg.IpgError) as e:
        g.run("sssp", source=100)
    assert e.value.status == ipg.EINVAL
    # bad graphs are caught by device-side validation
    off = torch.tensor([0, 2, 1, 3], dtype=torch.int64, device="cuda")
    dst = torch.tensor([1, 2, 0], dtype=torch.int32, device="cuda")
    with pytest.raises(ipg.IpgError) as e:
        ipg.Graph(3, off, dst, off, dst, symmetric=True)
    assert e.value.status == ipg.EBADGRAPH
    off = torch.tensor([0, 1, 2, 3], dtype=torch.int64, device="cuda")
    dst = torch.tensor([1, 2, 3], dtype=torch.int32, device="cuda")
    with pytest.raises(ipg.IpgError) as e:
        ipg.Graph(3, off, dst, off, dst, symmetric=True)
    assert e.value.status == ipg.EBADGRAPH
    dst = torch.tensor([1, 2, -1], dtype=torch.int32, device="cuda")
    with pytest.raises(ipg.IpgError) as e:
        ipg.Graph(3, off, dst, off, dst, symmetric=True)
    assert e.value.status == ipg.EBADGRAPH
    off = torch.tensor([0, 1, 2, 4], dtype=torch.int64, device="cuda")
    dst = torch.tensor([1, 2, 0], dtype=torch.int32, device="cuda")
    with pytest.raises(ipg.IpgError):
        ipg.Graph(3, off, dst, off, dst, symmetric=True)


def test_sssp_overflow_reported(ipg):
    import torch

    hg = graphgen.from_edges(3, [0, 1], [1, 2])
    w = np.array([0xFFFFFFF0, 0x20], dtype=np.uint32)
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a).view(dt)).cuda()
    off = t(hg.csr_off.astype(np.uint64), np.int64)
    dst = t(hg.csr_dst, np.int32)
    coff = t(hg.csc_off.astype(np.uint64), np.int64)
    csrc = t(hg.csc_src, np.int32)
    ww = t(w, np.int32)
    cw = t(w[[0, 1]], np.int32)  # CSC order of this 2-edge path equals CSR order
    g = ipg.Graph(3, off, dst, coff, csrc, ww, cw)
    for mode in ("push", "pull"):
        with pytest.raises(ipg.IpgError) as e:
            g.run("sssp", source=0, mode=mode)
        assert e.value.status == ipg.EOVERFLOW


def test_small_workspace_rejected(ipg):
    import ctypes

    hg = random_graph(100, 300, seed=1)
    g = ipg.Graph.from_host(hg)
    rc = ipg.lib().ipg_run(g._h, 1, 1, 0, None, None, 0, None, None)
    assert rc == ipg.EWORKSPACE
    ws, nbytes = g.workspace(1)
    rc = ipg.lib().ipg_run(g._h, 1, 1, 0, None, ws.data_ptr(), nbytes - 1, None, None)
    assert rc == ipg.EWORKSPACE


def test_push_hub_senders(ipg):
    # Senders with many out-edges queue them as pieces that a second launch
    # spreads over the grid; degrees far above the piece size, several such
    # senders in one superstep, and such senders reached in later supersteps.
    rng = np.random.default_rng(5)
    n = 60000
    src, dst = [], []
    for c, d in ((0, 8191), (1, 8192), (2, 20000), (3, 30000)):
        leaves = rng.choice(np.arange(10, n), size=d, replace=False)
        src += [c] * d
        dst += leaves.tolist()
    src += rng.integers(4, n, size=40000).tolist()
    dst += rng.integers(4, n, size=40000).tolist()
    hg = graphgen.from_edges(n, np.array(src), np.array(dst), symmetric=True, name="hubs")
    assert (np.diff(hg.csr_off) >= 8192).sum() >= 3
    for app, source in (("cc", 0), ("sssp", 2), ("sssp", 12345)):
        check_min_app(ipg, hg, app, source=source)
        ref = oracle.run_graph(app, hg, 0, source=source)
        g = ipg.Graph.from_host(hg)
        vals, st = g.run(app, source=source, mode="push", persistent=True)
        assert np.array_equal(to_np(vals), ref.values) and np.array_equal(st.trace, ref.trace)


@pytest.mark.parametrize("sym", [False, True])
def test_pagerank_hot_first_store(ipg, sym):
    # The renamed store (vertices renamed by descending out-degree, the CSC
    # rebuilt under the new names) sums the same values per row; only the
    # grouping of rows into work items changes, so ranks agree with the
    # oracle and with the plain store within the PageRank tolerance, and
    # the renamed runs are deterministic.
    import torch

    hg = graphgen.rmat(15, 16, seed=8, symmetric=sym)
    a = ipg.Graph.from_host(hg, rename=True)
    b = ipg.Graph.from_host(hg, rename=False)
    for T in (0, 1, 10):
        ref = oracle.run_graph("pagerank", hg, T)
        ra, _ = a.run("pagerank", T, mode="pull")
        rb, _ = b.run("pagerank", T, mode="pull")
        assert max_rel(to_np(ra), ref.values) <= PR_RTOL and max_rel(to_np(rb), ref.values) <= PR_RTOL
        assert torch.equal(ra, a.run("pagerank", T, mode="pull")[0])
    d = oracle.pagerank_deltas(hg.n, hg.csr_off, hg.csr_dst, 200)
    tol = 1e-9
    while np.any(np.abs(d[1:] - tol) <= max(1e-6 * tol, 1e-12)):
        tol *= 1.37
    ref, T, _ = oracle.pagerank_converge(hg, tol, 200)
    ca, sa = a.run("pagerank", 200, mode="pull", tol=tol)
    assert sa.supersteps == T + 1 and max_rel(to_np(ca), ref.values) <= PR_RTOL
    # parts: each part's N, under the new names
    parts = torch.tensor([0, 1000, hg.n], dtype=torch.int32, device="cuda")
    pa, _ = a.run("pagerank", 5, parts=parts)
    pb, _ = b.run("pagerank", 5, parts=parts)
    assert max_rel(to_np(pa), to_np(pb)) <= PR_RTOL
    # graph replay of the renamed run
    assert torch.equal(a.run("pagerank", 10, mode="pull", graph=True)[0], a.run("pagerank", 10, mode="pull")[0])
    # CC and SSSP read the caller's CSC either way
    for app in ("cc", "sssp"):
        assert torch.equal(a.run(app)[0], b.run(app)[0])


def test_launch_parameters_never_change_results(ipg):
    # every point of the autotuner's search space: PageRank within the
    # tolerance of the oracle, CC / SSSP / batched SSSP exact
    from paper_2010_08781_amd import autotune

    hg = graphgen.rmat(15, 16, seed=9, symmetric=True)
    g = ipg.Graph.from_host(hg)
    ref = oracle.run_graph("pagerank", hg, 10)
    for hot in autotune.SPACES["pagerank"]["pr_hot"]:
        for grid in (64, 1024, 4096):
            r, _ = g.run("pagerank", 10, mode="pull", tuning={"pr_hot": hot, "pull_grid": grid})
            assert max_rel(to_np(r), ref.values) <= PR_RTOL, (hot, grid)
    for app in ("cc", "sssp"):
        ref = oracle.run_graph(app, hg, 0, source=0)
        for t in ({"push_div": 10, "list_div": 8, "pull_grid": 64}, {"push_div": 40, "list_div": 32},
                  {"push_div": 1}, {"push_div": 100000, "gate_div": 1}, {"push_div": 100000, "gate_div": 0xFFFFFFFF},
                  {"gate_div": 2, "pull_grid": 100}):
            for persistent in (False, True):
                v, st = g.run(app, tuning=t, persistent=persistent)
                assert np.array_equal(to_np(v), ref.values) and np.array_equal(st.trace, ref.trace), (app, t)
    src = graphgen.pick_sources(hg, 40, seed=1)
    want = g.run_multi_sssp(src)[0]
    for t in ({"push_div": 5, "pull_grid": 64}, {"push_div": 40, "pull_grid": 4096}):
        assert np.array_equal(g.run_multi_sssp(src, tuning=t)[0].cpu().numpy(), want.cpu().numpy())


def test_autotune_on_device(ipg, tmp_path):
    from paper_2010_08781_amd import autotune

    hg = graphgen.rmat(14, 16, seed=1)
    g = ipg.Graph.from_host(hg)
    best = autotune.tune(g, hg, "pagerank", cache_path=str(tmp_path / "t.json"), reps=1)
    r, _ = g.run("pagerank", 10, tuning=best)
    assert max_rel(to_np(r), oracle.run_graph("pagerank", hg, 10).values) <= PR_RTOL
    best = autotune.tune(g, hg, "sssp", cache_path=str(tmp_path / "t.json"), reps=1)
    assert set(best) == {"push_div", "list_div", "pull_grid", "gate_div", "late_div"}
