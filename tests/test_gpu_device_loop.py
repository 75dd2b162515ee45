"""GPU parity of the device-driven superstep loop (IPG_RUN_PERSISTENT).

The control block on the device takes the host loop's decisions (halt, cap,
overflow, active set, exchange), so values, traces and superstep counts must
equal the oracle's exactly, for every exchange policy, and agree with the
host-driven loop superstep by superstep -- including the exchange chosen.
"""
import numpy as np
import pytest

import graphgen
import oracle
from oracle import mlp
from tests.graphs_small import path, random_graph

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ipg():
    import torch

    import paper_2010_08781_amd as m

    assert torch.cuda.is_available()
    m.lib()
    return m


def check(ipg, hg, app, source=0, modes=("auto", "push", "pull"), selector=None):
    ref = oracle.run_graph(app, hg, 0, source=source)
    assert ref.status == oracle.OK
    g = ipg.Graph.from_host(hg)
    for mode in modes:
        print(f"[device-loop] {hg.name} {app} src={source} mode={mode}", flush=True)
        vals, st = g.run(app, source=source, mode=mode, persistent=True, selector=selector)
        got = ipg.values_to_numpy(vals)
        assert np.array_equal(got, ref.values), f"{app} {mode}: {np.sum(got != ref.values)} values differ"
        assert st.supersteps == ref.supersteps
        assert np.array_equal(st.trace, ref.trace), f"{app} {mode}\n{st.trace}\n{ref.trace}"
        assert st.halted and st.status == ipg.OK
        assert st.edges_traversed == int(ref.trace[:, 2].sum())
        # the host-driven loop takes the same decisions
        _, sh = g.run(app, source=source, mode=mode, selector=selector)
        assert np.array_equal(sh.mode, st.mode)
        assert np.array_equal(sh.examined, st.examined)
        assert (st.usec > 0).all()
    return g


@pytest.mark.parametrize("app", ["cc", "sssp"])
def test_rmat_s16_symmetrised(ipg, app):
    check(ipg, graphgen.rmat(16, 16, seed=6, symmetric=True), app)


def test_rmat_s14_directed(ipg):
    hg = graphgen.rmat(14, 16, seed=1, symmetric=False)
    check(ipg, hg, "cc")
    check(ipg, hg, "sssp", source=int(graphgen.pick_sources(hg, 1, seed=3)[0]))


def test_weighted_grid_with_shortcuts(ipg):
    # the persistent-path workload in miniature: weighted, high diameter
    check(ipg, graphgen.grid_with_shortcuts(256, 0.01, seed=3), "sssp")


def test_long_path_many_chunks(ipg):
    # 600 supersteps: chunks grow to their maximum and the run halts inside one
    check(ipg, path(599), "sssp", modes=("auto", "push"))
    check(ipg, path(300), "cc", modes=("auto",))


def test_weighted_directed_loops_dups(ipg):
    check(ipg, random_graph(3000, 20000, seed=10, loops=True, dups=True, weight_seed=3), "sssp", source=5)


def test_selector_drives_device_loop(ipg):
    import torch

    hg = graphgen.rmat(14, 16, seed=3, symmetric=True)
    for seed in (9, 11):
        p = torch.tensor(mlp.init_params(seed, scale=3.0), dtype=torch.float64, device="cuda")
        check(ipg, hg, "cc", modes=("auto",), selector=p)
        check(ipg, hg, "sssp", modes=("auto",), selector=p)


def test_first_chunk_from_previous_run(ipg):
    # A run's first chunk is the previous device-driven run's superstep count
    # for that application on the handle.  A long run (300 supersteps along a
    # path) followed by short ones -- from the path's middle, and from an
    # isolated vertex (one superstep), where most of the first chunk's
    # supersteps return at once -- and a long one again, each matching the
    # oracle; then a cap below the guessed chunk.
    n = 300
    hg = graphgen.from_edges(n + 1, np.arange(n - 1), np.arange(1, n), symmetric=True, name="path+isolated")  # vertex n: isolated
    g = ipg.Graph.from_host(hg)
    for source in (0, n // 2, n, 0, n):
        ref = oracle.run_graph("sssp", hg, 0, source=source)
        vals, st = g.run("sssp", source=source, mode="auto", persistent=True)
        assert np.array_equal(ipg.values_to_numpy(vals), ref.values), source
        assert st.supersteps == ref.supersteps and np.array_equal(st.trace, ref.trace), source
    ref = oracle.run_graph("cc", hg, 0)
    for _ in range(2):
        vals, st = g.run("cc", persistent=True)
        assert np.array_equal(ipg.values_to_numpy(vals), ref.values) and st.supersteps == ref.supersteps
    g.run("sssp", source=0, persistent=True)  # the next guess: 300 supersteps, capped to a chunk of 64
    ref = oracle.run_graph("sssp", hg, 5, source=0)
    vals, st = g.run("sssp", 5, source=0, persistent=True)
    assert st.status == ipg.NOT_CONVERGED and st.supersteps == 5 and not st.halted
    assert np.array_equal(ipg.values_to_numpy(vals), ref.values) and np.array_equal(st.trace, ref.trace)


def test_cap_and_overflow(ipg):
    import torch

    hg = path(50)
    g = ipg.Graph.from_host(hg)
    ref = oracle.run_graph("cc", hg, 7)
    vals, st = g.run("cc", 7, persistent=True)
    assert st.status == ipg.NOT_CONVERGED and st.supersteps == 7 and not st.halted
    assert np.array_equal(ipg.values_to_numpy(vals), ref.values)
    assert np.array_equal(st.trace, ref.trace)
    # an SSSP message that would reach INF
    hg = graphgen.from_edges(3, [0, 1], [1, 2])
    w = np.array([0xFFFFFFF0, 0x20], dtype=np.uint32)
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a).view(dt)).cuda()
    off, dst = t(hg.csr_off.astype(np.uint64), np.int64), t(hg.csr_dst, np.int32)
    coff, csrc = t(hg.csc_off.astype(np.uint64), np.int64), t(hg.csc_src, np.int32)
    g = ipg.Graph(3, off, dst, coff, csrc, t(w, np.int32), t(w, np.int32))
    for mode in ("push", "pull", "auto"):
        with pytest.raises(ipg.IpgError) as e:
            g.run("sssp", source=0, mode=mode, persistent=True)
        assert e.value.status == ipg.EOVERFLOW


def test_edge_cases(ipg):
    check(ipg, graphgen.from_edges(1, [], []), "cc")
    check(ipg, graphgen.from_edges(4, [], []), "sssp", source=3)
    check(ipg, random_graph(200, 50, seed=2), "cc")
