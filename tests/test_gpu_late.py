"""GPU parity of the late push (ipg_tuning.late_div): a CC/SSSP superstep
chosen as pull whose broadcasts, counted after its compute, carry few
messages is exchanged by push instead (Section 4.3.2's push/pull choice,
taken on the messages themselves).

The exchange never changes values or traces (Figs. 9, 10 with the min
combiner), so every run must equal the oracle exactly.  Cases: late_div = 1
(every pull superstep after the first turns to a push), the default and
never; both loops (which must take the same decisions superstep by
superstep); the plain store (row-item pull), the blocked store, the binned
store (cold sources in slots) and a weighted graph; forced pull stays pull.
"""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

NEVER = 0xFFFFFFFF
PUSH, PULL = 1, 2


@pytest.fixture(scope="module")
def ipg():
    import torch

    import paper_2010_08781_amd as m

    assert torch.cuda.is_available()
    m.lib()
    return m


def runs(ipg, g, hg, app, source, weighted=True):
    """Runs every late_div on both loops against the oracle; returns the
    modes per late_div (device loop)."""
    ref = oracle.run_graph(app, hg, 0, source=source, weighted=weighted)
    assert ref.status == oracle.OK
    modes = {}
    for late in (1, 0, NEVER):
        tuning = {"late_div": late} if late else None
        got = {}
        for persistent in (False, True):
            print(f"[late] {hg.name} {app} src={source} late_div={late} persistent={persistent}", flush=True)
            vals, st = g.run(app, source=source, mode="auto", persistent=persistent, tuning=tuning)
            assert np.array_equal(ipg.values_to_numpy(vals), ref.values), (app, late, persistent)
            assert st.supersteps == ref.supersteps and st.halted
            assert np.array_equal(st.trace, ref.trace), (app, late, persistent)
            assert st.edges_traversed == int(ref.trace[:, 2].sum())
            # a push reads exactly the messages' edges, a pull every in-edge
            msgs = np.asarray(ref.trace[:, 2], dtype=np.uint64)
            push = st.mode == PUSH
            assert np.array_equal(st.examined[push], msgs[push])
            assert (st.examined[~push] == hg.m).all()
            got[persistent] = (st.mode.copy(), st.examined.copy())
        # the host-driven loop takes the device-driven loop's decisions
        assert np.array_equal(got[False][0], got[True][0]), (app, late, got)
        assert np.array_equal(got[False][1], got[True][1]), (app, late)
        modes[late] = got[True][0]
    # every superstep >= 1 that the rule pulls is a late push at late_div = 1
    never = modes[NEVER]
    assert (modes[1][1:] == PUSH).all(), modes
    # late pushes only replace pulls
    assert ((modes[0] == never) | ((never == PULL) & (modes[0] == PUSH))).all()
    return modes


def forced_pull_stays(ipg, g, hg, app, source):
    ref = oracle.run_graph(app, hg, 0, source=source)
    for persistent in (False, True):
        vals, st = g.run(app, source=source, mode="pull", persistent=persistent, tuning={"late_div": 1})
        assert np.array_equal(ipg.values_to_numpy(vals), ref.values)
        assert (st.mode == PULL).all() and (st.examined == hg.m).all()


@pytest.mark.parametrize("app", ["cc", "sssp"])
def test_plain_store(ipg, app):
    hg = graphgen.rmat(16, 16, seed=6, symmetric=True)
    g = ipg.Graph.from_host(hg)
    modes = runs(ipg, g, hg, app, 0)
    assert (modes[NEVER][1:] == PULL).any(), "the case should pull at least once after superstep 0"
    forced_pull_stays(ipg, g, hg, app, 0)


@pytest.mark.parametrize("app", ["cc", "sssp"])
def test_blocked_store(ipg, app):
    hg = graphgen.rmat(17, 16, seed=8, symmetric=True)
    g = ipg.Graph.from_host(hg, blocked=True)
    runs(ipg, g, hg, app, 0)
    forced_pull_stays(ipg, g, hg, app, 0)


@pytest.mark.parametrize("app", ["cc", "sssp"])
def test_binned_store(ipg, app):
    # sources from 16384 on binned: cold chunks read slots
    hg = graphgen.rmat(16, 16, seed=9, symmetric=True)
    g = ipg.Graph.from_host(hg, blocked=True, binned=True, binned_hot=16384)
    runs(ipg, g, hg, app, 0)


def test_directed_and_weighted(ipg):
    hg = graphgen.rmat(14, 16, seed=1, symmetric=False)
    g = ipg.Graph.from_host(hg)
    runs(ipg, g, hg, "cc", 0)
    runs(ipg, g, hg, "sssp", int(graphgen.pick_sources(hg, 1, seed=3)[0]))
    # weighted, high diameter: the row-item pull with CSC weights, the late push with CSR weights
    hg = graphgen.grid_with_shortcuts(256, 0.01, seed=3)
    g = ipg.Graph.from_host(hg)
    runs(ipg, g, hg, "sssp", 0)


def test_edge_cases(ipg):
    from tests.graphs_small import path, random_graph

    for hg, app in ((graphgen.from_edges(4, [], []), "cc"), (random_graph(200, 50, seed=2), "cc"),
                    (path(40), "sssp"), (random_graph(3000, 20000, seed=10, loops=True, dups=True), "cc")):
        g = ipg.Graph.from_host(hg)
        runs(ipg, g, hg, app, 0)


@pytest.mark.parametrize("app", ["cc", "sssp"])
def test_push_variants_of_the_selector(ipg, app):
    # The variants the selector scores, forced as its training forces them:
    # every push over the list (list_div = 1), every push sweeping the
    # mailboxes (list_div = UINT32_MAX), every pull -- same values and trace,
    # on the caller's names (directed) and under the hot-first names
    # (symmetric, blocked), in both loops.
    for hg in (graphgen.rmat(15, 16, seed=12, symmetric=True), graphgen.rmat(14, 16, seed=13)):
        ref = oracle.run_graph(app, hg, 0, source=0)
        g = ipg.Graph.from_host(hg, blocked=True)
        for mode, tuning in (("push", {"list_div": 1}), ("push", {"list_div": NEVER}), ("pull", None)):
            for persistent in (False, True):
                v, st = g.run(app, source=0, mode=mode, tuning=tuning, persistent=persistent)
                assert np.array_equal(ipg.values_to_numpy(v), ref.values), (hg.name, mode, tuning, persistent)
                assert np.array_equal(st.trace, ref.trace), (hg.name, mode, tuning, persistent)
