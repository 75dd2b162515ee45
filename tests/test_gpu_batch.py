"""GPU parity of the batched forms against the oracle, through the C ABI.

Batched SSSP (ipg_run_multi_sssp): row i of the [Q, N] result equals the
oracle's single-source SSSP from sources[i], bit for bit, and the batched
trace equals the sum over queries of the oracle's single-source traces
(a query that has halted adds zeros); the superstep count is the largest of
the queries'.  The exchange (push, pull, per-superstep choice) never
changes any of it.
"""
import numpy as np
import pytest

import graphgen
import oracle
from tests.graphs_small import path, random_graph

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ipg():
    import torch

    import paper_2010_08781_amd as m

    assert torch.cuda.is_available()
    m.lib()
    return m


def oracle_batch(hg, sources):
    """Single-source oracle runs: values [Q, N] and the summed, zero-padded trace."""
    runs = [oracle.run_graph("sssp", hg, 0, source=int(s)) for s in sources]
    for r in runs:
        assert r.status == oracle.OK
    S = max(r.supersteps for r in runs)
    tr = np.zeros((S, 3), dtype=np.uint64)
    for r in runs:
        tr[: r.supersteps] += r.trace.astype(np.uint64)
    return np.stack([r.values for r in runs]), tr, S


def check_batch(ipg, hg, sources, modes=("auto", "push", "pull")):
    vals, tr, S = oracle_batch(hg, sources)
    g = ipg.Graph.from_host(hg)
    for mode in modes:
        print(f"[batch] {hg.name} Q={len(sources)} mode={mode}", flush=True)
        d, st = g.run_multi_sssp(sources, mode=mode)
        got = d.cpu().numpy().view(np.uint32)
        bad = np.argwhere(got != vals)
        assert bad.size == 0, f"{mode}: {len(bad)} distances differ, first (query, vertex) {bad[:5].tolist()}"
        assert st.supersteps == S, (mode, st.supersteps, S)
        assert np.array_equal(st.trace, tr), f"{mode} trace\n{st.trace}\n{tr}"
        assert st.halted
        assert st.edges_traversed == int(tr[:, 2].sum())
    return g


@pytest.mark.parametrize("q", [1, 7, 64, 65, 130, 256])
def test_batch_rmat_sym(ipg, q):
    hg = graphgen.rmat(12, 16, seed=7, symmetric=True)
    src = graphgen.pick_sources(hg, q, seed=100 + q)
    check_batch(ipg, hg, src)


def test_batch_rmat_directed_with_hubs(ipg):
    # s14 directed: in-degree hubs above the long-row threshold, vertices
    # without in-edges, sources whose reach is a small part of the graph
    hg = graphgen.rmat(14, 16, seed=1, symmetric=False)
    assert (np.diff(hg.csc_off) > 256).any()
    src = graphgen.pick_sources(hg, 96, seed=5)
    check_batch(ipg, hg, src)


def test_batch_repeated_and_isolated_sources(ipg):
    # repeated sources, a source without out-edges, a self-loop and duplicate edges
    hg = random_graph(300, 900, seed=3, loops=True, dups=True)
    deg = np.diff(hg.csr_off)
    sink = int(np.flatnonzero(deg == 0)[0]) if (deg == 0).any() else 0
    src = np.array([0, 5, 5, sink, 17, 0, 299] * 9, dtype=np.uint32)
    check_batch(ipg, hg, src)


def test_batch_long_path(ipg):
    # many supersteps with one-vertex frontiers, push and pull alternating
    hg = path(400)
    check_batch(ipg, hg, np.array([0, 399, 200, 1], dtype=np.uint32))


def test_batch_star_hub(ipg):
    # one vertex with in- and out-degree far above the chunk size
    n = 5000
    leaves = np.arange(1, n)
    hg = graphgen.from_edges(n, np.zeros(n - 1, dtype=np.int64), leaves, symmetric=True, name="star")
    check_batch(ipg, hg, np.array([0, 1, 4999, 77], dtype=np.uint32))


def test_batch_single_vertex_and_no_edges(ipg):
    hg = graphgen.from_edges(5, np.array([], dtype=np.int64), np.array([], dtype=np.int64), name="empty5")
    check_batch(ipg, hg, np.array([0, 4, 2], dtype=np.uint32))


def test_batch_cap_not_converged(ipg):
    hg = path(50)
    g = ipg.Graph.from_host(hg)
    d, st = g.run_multi_sssp([0, 10], max_supersteps=5)
    assert st.status == ipg.NOT_CONVERGED and st.supersteps == 5 and not st.halted
    got = d.cpu().numpy().view(np.uint32)
    want0 = np.where(np.arange(50) <= 4, np.arange(50), ipg.INF)
    assert np.array_equal(got[0], want0)


def test_batch_errors(ipg):
    import torch

    hg = random_graph(100, 300, seed=4)
    g = ipg.Graph.from_host(hg)
    with pytest.raises(ipg.IpgError) as e:
        g.run_multi_sssp(np.arange(257) % 100)
    assert e.value.status == ipg.EINVAL
    with pytest.raises(ipg.IpgError) as e:
        g.run_multi_sssp([3, 100])
    assert e.value.status == ipg.EINVAL
    with pytest.raises(ipg.IpgError) as e:
        g.run_multi_sssp(torch.zeros(0, dtype=torch.int32, device="cuda"))
    assert e.value.status == ipg.EINVAL
    hw = random_graph(100, 300, seed=4, weight_seed=9)
    gw = ipg.Graph.from_host(hw)
    with pytest.raises(ipg.IpgError) as e:
        gw.run_multi_sssp([0])
    assert e.value.status == ipg.EUNSUPPORTED


def test_batch_full_size_sampled(ipg):
    # The batched workload at full size: 256 sources on R-MAT scale 22
    # (symmetrised, edge factor 16).  Sampled queries against the oracle,
    # and the summed trace's invariants for all of them.
    hg = graphgen.workload("rmat-s22-sym")
    src = graphgen.pick_sources(hg, 256, seed=40)
    g = ipg.Graph.from_host(hg)
    print(f"[batch] rmat-s22-sym n={hg.n} m={hg.m} Q=256", flush=True)
    d, st = g.run_multi_sssp(src)
    assert st.halted
    deg = np.diff(hg.csr_off).astype(np.uint64)
    tr = st.trace
    assert tr[0, 0] == 256 * hg.n and tr[0, 1] == 256 and tr[0, 2] == int(deg[src].sum())
    for i in (0, 101, 255):
        ref = oracle.run_graph("sssp", hg, 0, source=int(src[i]))
        got = d[i].cpu().numpy().view(np.uint32)
        assert np.array_equal(got, ref.values), f"query {i}"
        assert ref.supersteps <= st.supersteps
    # every distance set is one sender in exactly one superstep: the number of
    # (query, vertex) pairs at distance s is senders(s)
    import torch

    per_level = torch.zeros(st.supersteps + 1, dtype=torch.int64, device="cuda")
    for i in range(256):
        row = d[i].to(torch.int64) & 0xFFFFFFFF
        row = row[row != ipg.INF]
        assert int(row.max()) < st.supersteps
        per_level += torch.bincount(row, minlength=st.supersteps + 1)
    assert np.array_equal(per_level.cpu().numpy()[: st.supersteps].astype(np.uint64), tr[:, 1])


# --------------------------------------------------- PageRank over parts --
#
# A disjoint union of graphs with per-part N: each part's ranks equal a
# separate oracle run on that part (within the PageRank tolerance), in both
# exchanges, eagerly and replayed as a hipGraph.

PR_RTOL = 1e-12


def _parts_tensor(u):
    import torch

    return torch.from_numpy(u.meta["parts"].astype(np.int32)).cuda()


def _check_parts(u, graphs, ranks, T):
    r = ranks.cpu().numpy()
    offs = u.meta["parts"].astype(np.int64)
    for i, hg in enumerate(graphs):
        ref = oracle.run_graph("pagerank", hg, T)
        got = r[offs[i]: offs[i + 1]]
        err = float(np.max(np.abs(got - ref.values) / np.abs(ref.values)))
        assert err <= PR_RTOL, f"part {i} (n={hg.n}): max rel err {err:.3e}"


def test_pagerank_parts_match_separate_runs(ipg):
    graphs = [graphgen.rmat_small(n, 8, seed=200 + n) for n in (1000, 1500, 3000, 64, 5000, 777)]
    graphs.append(random_graph(50, 200, seed=9, loops=True, dups=True))
    u = graphgen.disjoint_union(graphs)
    g = ipg.Graph.from_host(u)
    parts = _parts_tensor(u)
    for mode in ("pull", "push"):
        for T in (0, 1, 20):
            ranks, st = g.run("pagerank", T, mode=mode, parts=parts)
            _check_parts(u, graphs, ranks, T)
            assert st.supersteps == T + 1


def test_pagerank_graph_replay_equals_eager(ipg):
    import torch

    graphs = [graphgen.rmat_small(n, 8, seed=300 + n) for n in (2000, 4000, 1024)]
    u = graphgen.disjoint_union(graphs)
    g = ipg.Graph.from_host(u)
    parts = _parts_tensor(u)
    eager = {T: g.run("pagerank", T, mode="pull", parts=parts)[0].clone() for T in (5, 20)}
    for rep in range(4):
        for T in (20, 20, 5):  # same key replays; a new T re-captures
            r, st = g.run("pagerank", T, mode="pull", parts=parts, graph=True)
            assert torch.equal(r, eager[T]), f"replay {rep} T={T}"
            assert st.seconds > 0
        # eager work and synchronisation between replays
        g.run("cc")
        torch.cuda.synchronize()
    r, _ = g.run("pagerank", 20, mode="push", parts=parts, graph=True)
    _check_parts(u, graphs, r, 20)
    # a whole graph (no parts) replayed
    r, _ = g.run("pagerank", 7, mode="pull", graph=True)
    assert torch.equal(r, g.run("pagerank", 7, mode="pull")[0])


def test_pagerank_parts_errors(ipg):
    import torch

    u = graphgen.disjoint_union([random_graph(30, 90, seed=1), random_graph(20, 60, seed=2)])
    g = ipg.Graph.from_host(u)
    for bad in ([0, 30, 49], [0, 30, 30, 50], [1, 30, 50]):
        with pytest.raises(ipg.IpgError) as e:
            g.run("pagerank", 3, parts=torch.tensor(bad, dtype=torch.int32, device="cuda"))
        assert e.value.status == ipg.EINVAL
    with pytest.raises(ipg.IpgError) as e:
        g.run("cc", parts=_parts_tensor(u))
    assert e.value.status == ipg.EUNSUPPORTED
    with pytest.raises(ipg.IpgError) as e:
        g.run("sssp", graph=True)
    assert e.value.status == ipg.EUNSUPPORTED


def test_pagerank_small_graph_family_full_size(ipg):
    # The batched workload at full size: 64 directed R-MAT graphs, n
    # log-uniform in [2^10, 2^16], edge factor 8, 20 updates, one graph launch.
    graphs = graphgen.small_graph_family(64, seed=41)
    u = graphgen.disjoint_union(graphs, name="family64")
    g = ipg.Graph.from_host(u)
    print(f"[batch] family64 n={u.n} m={u.m}", flush=True)
    r, st = g.run("pagerank", 20, mode="pull", parts=_parts_tensor(u), graph=True)
    _check_parts(u, graphs, r, 20)


# ------------------------------------------ device-driven and one launch --

@pytest.mark.parametrize("case", ["rmat", "path", "dir"])
def test_batch_device_driven_matches_oracle(ipg, case):
    # the superstep loop on the device (control block, chunks of 16
    # supersteps with the level ring expanded after each chunk)
    if case == "rmat":
        hg = graphgen.rmat(12, 16, seed=7, symmetric=True)
        src = graphgen.pick_sources(hg, 130, seed=3)
    elif case == "path":
        hg = path(400)  # about 400 supersteps: many chunks and ring wraps
        src = np.array([0, 399, 200, 1], dtype=np.uint32)
    else:
        hg = graphgen.rmat(14, 16, seed=1, symmetric=False)
        src = graphgen.pick_sources(hg, 96, seed=5)
    vals, tr, S = oracle_batch(hg, src)
    g = ipg.Graph.from_host(hg)
    for mode in ("auto", "push", "pull"):
        d, st = g.run_multi_sssp(src, mode=mode, persistent=True)
        assert np.array_equal(d.cpu().numpy().view(np.uint32), vals), mode
        assert st.supersteps == S and st.halted and np.array_equal(st.trace, tr), mode
        assert st.seconds > 0 and (st.usec > 0).all()


def test_batch_enqueue_then_result(ipg):
    import torch

    hg = graphgen.rmat(12, 16, seed=9, symmetric=True)
    src = graphgen.pick_sources(hg, 64, seed=2)
    vals, tr, S = oracle_batch(hg, src)
    g = ipg.Graph.from_host(hg)
    d, st = g.run_multi_sssp(src, max_supersteps=64, enqueue=True)
    assert st is None
    st = g.multi_sssp_result()
    assert st.status == ipg.OK and st.supersteps == S and np.array_equal(st.trace, tr)
    assert np.array_equal(d.cpu().numpy().view(np.uint32), vals)
    # capped before the end: the distances set so far, the rest INF
    d, _ = g.run_multi_sssp(src, max_supersteps=3, enqueue=True)
    st = g.multi_sssp_result()
    assert st.status == ipg.NOT_CONVERGED and st.supersteps == 3 and not st.halted
    got = d.cpu().numpy().view(np.uint32)
    assert np.array_equal(got, np.where(vals <= 2, vals, ipg.INF))
    with pytest.raises(ipg.IpgError) as e:
        g.run_multi_sssp(src, max_supersteps=0, enqueue=True)
    assert e.value.status == ipg.EINVAL
    # an out-of-range source is skipped on the device and reported afterwards
    bad = torch.tensor([0, hg.n + 5, 3], dtype=torch.int32, device="cuda")
    g.run_multi_sssp(bad, max_supersteps=64, enqueue=True)
    with pytest.raises(ipg.IpgError) as e:
        g.multi_sssp_result()
    assert e.value.status == ipg.EINVAL


def test_batch_plan_is_one_graph_launch(ipg):
    # batched SSSP + PageRank over a union of graphs captured as one graph;
    # every replay, with eager work and synchronisation in between, equals
    # the eager runs and the oracle
    import torch

    from paper_2010_08781_amd.batch import BatchPlan

    hs = graphgen.rmat(13, 16, seed=11, symmetric=True)
    src = graphgen.pick_sources(hs, 200, seed=4)
    vals, tr, S = oracle_batch(hs, src)
    fam = [graphgen.rmat_small(n, 8, seed=600 + n) for n in (1024, 3000, 1500, 5000)]
    u = graphgen.disjoint_union(fam)
    gs, gp = ipg.Graph.from_host(hs), ipg.Graph.from_host(u)
    parts = torch.from_numpy(u.meta["parts"].astype(np.int32)).cuda()
    eager_ranks = gp.run("pagerank", 20, mode="pull", parts=parts)[0].clone()
    plan = BatchPlan(gs, src, gp, parts, updates=20, max_supersteps=48).capture()
    offs = u.meta["parts"].astype(np.int64)
    refs = [oracle.run_graph("pagerank", h, 20).values for h in fam]
    for rep in range(3):
        plan.dist.fill_(0)
        plan.replay()
        d, st = plan.sssp()
        assert np.array_equal(d.cpu().numpy().view(np.uint32), vals), rep
        assert st.supersteps == S and np.array_equal(st.trace, tr), rep
        r = plan.ranks()
        assert torch.equal(r, eager_ranks), rep
        rn = r.cpu().numpy()
        for i, ref in enumerate(refs):
            assert np.max(np.abs(rn[offs[i]: offs[i + 1]] - ref) / ref) <= 1e-12
        gs.run("cc")  # eager work between replays
        torch.cuda.synchronize()
