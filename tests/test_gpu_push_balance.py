"""GPU parity of the push exchange's load balancing and segmented queues.

A sender with at least 128 out-edges queues its out-edges as pieces of up to
1024 edges, which a second launch deals over the grid; the queue and the
next-frontier list are cut into 64 segments, one per counter slot.  A piece
segment that is full sends its sender back to in-place expansion, and a full
list segment drops the list (the next superstep sweeps the mailboxes).
Every case is compared with the oracle, values and traces bit-exact, with
the exchange forced to push in every superstep and in both loops.
"""
import numpy as np
import pytest

import graphgen
import oracle
from tests.graphs_small import random_graph

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ipg():
    import torch

    import paper_2010_08781_amd as m

    assert torch.cuda.is_available()
    m.lib()
    return m


def check(ipg, hg, app, source=0, weighted=True, modes=("push", "auto"), blocked=False):
    ref = oracle.run_graph(app, hg, 0, source=source, weighted=weighted)
    assert ref.status == oracle.OK
    g = ipg.Graph.from_host(hg, weighted=weighted, blocked=blocked)
    for mode in modes:
        for persistent in (False, True):
            vals, st = g.run(app, source=source, mode=mode, persistent=persistent)
            got = ipg.values_to_numpy(vals)
            assert np.array_equal(got, ref.values), (app, mode, persistent, int(np.sum(got != ref.values)))
            assert np.array_equal(st.trace, ref.trace), (app, mode, persistent)
            assert st.halted


def star(n, extra=0, seed=0):
    # center 0 linked to every other vertex, plus random edges among the leaves
    rng = np.random.default_rng(seed)
    src = np.concatenate([np.zeros(n - 1, np.int64), rng.integers(1, n, extra)])
    dst = np.concatenate([np.arange(1, n), rng.integers(1, n, extra)])
    return graphgen.from_edges(n, src, dst, symmetric=True)


@pytest.mark.parametrize("n", [130, 1100, 5000, 40000])
def test_star_pieces_fit(ipg, n):
    # the center's out-edges: one piece (130) up to 40 pieces, dealt over the grid
    hg = star(n, extra=8 * n, seed=n)
    for app, src in (("sssp", 0), ("sssp", 7), ("cc", 0)):
        check(ipg, hg, app, source=src)


def test_star_pieces_overflow_and_list_overflow(ipg):
    # E = 300K (both directions): a segment of the piece queue holds
    # (E/1024 + E/128)/64 + 64 = 105 pieces, fewer than the center's 147, so
    # the center is expanded in place by one workgroup, whose list segment
    # (N/64 + 64 = 2407 entries) then overflows: the next superstep sweeps
    # the mailboxes.
    hg = star(150000)
    for app, src in (("sssp", 0), ("sssp", 3), ("cc", 0)):
        check(ipg, hg, app, source=src)


@pytest.mark.parametrize("scale", [14, 17])
def test_rmat_low_id_hubs_forced_push(ipg, scale):
    # R-MAT puts its high-degree vertices at low ids: every dense push
    # superstep queues thousands of pieces from a few workgroups
    hg = graphgen.rmat(scale, 16, seed=40 + scale, symmetric=True)
    for app, src in (("cc", 0), ("sssp", 0), ("sssp", 999)):
        check(ipg, hg, app, source=src)


@pytest.mark.parametrize("app,src", [("sssp", 0), ("sssp", 7), ("cc", 0)])
def test_pieces_with_blocked_in_edges(ipg, app, src):
    # unit weights over blocked in-edges: in the device-driven loop a push
    # superstep's pieces run in the launch that is the blocked pull's second
    # launch in a pull superstep, and its push in the pull form's compute launch
    for hg in (star(5000, extra=40000, seed=3), graphgen.rmat(15, 16, seed=41, symmetric=True)):
        check(ipg, hg, app, source=src, weighted=False, blocked=True, modes=("push", "auto", "pull"))


def test_weighted_directed_multigraph_forced_push(ipg):
    check(ipg, graphgen.rmat(15, 16, seed=77, symmetric=False, weight_seed=5), "sssp", source=0, weighted=True)
    check(ipg, random_graph(3000, 200000, seed=8, loops=True, dups=True, weight_seed=9), "sssp", source=1, weighted=True)


def test_full_size_rmat_s20_forced_push(ipg):
    hg = graphgen.workload("rmat-s20-sym")
    check(ipg, hg, "cc", modes=("push",))
    check(ipg, hg, "sssp", source=0, modes=("push",))
