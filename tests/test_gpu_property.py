"""Property-based GPU parity (hypothesis): random small graphs -- any size
from one vertex, self-loops and duplicate edges kept or not, directed or
symmetrised, weighted or not -- run through the C ABI in every exchange,
both loops, on the plain and the blocked stores, against the oracle: CC and
SSSP values and traces bit-exact, PageRank within 1e-12 with its trace.
(The binned store needs more than 65536 vertices; its parity tests are the
blocked-store ones.)"""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from tests.graph_strategies import small_graphs

pytestmark = pytest.mark.gpu

SETTINGS = settings(max_examples=40, deadline=None, derandomize=True,
                    suppress_health_check=[HealthCheck.too_slow, HealthCheck.data_too_large,
                                           HealthCheck.function_scoped_fixture])


@pytest.fixture(scope="module")
def ipg():
    import torch

    import paper_2010_08781_amd as m

    assert torch.cuda.is_available()
    m.lib()
    return m


def max_rel(a, b):
    return float(np.max(np.abs(a - b) / np.abs(b))) if b.size else 0.0


@SETTINGS
@given(g=small_graphs(), store=st.sampled_from(["plain", "blocked"]))
def test_random_graphs_match_oracle(ipg, g, store):
    dev = ipg.Graph.from_host(g, rename=store != "plain", blocked=store != "plain")
    ref = oracle.run_graph("pagerank", g, 6)
    for mode in ("pull", "push"):
        vals, st_ = dev.run("pagerank", 6, mode=mode)
        assert max_rel(ipg.values_to_numpy(vals), ref.values) <= 1e-12, (store, mode)
        assert np.array_equal(st_.trace, ref.trace)
    for app in ("cc", "sssp"):
        src = g.n - 1 if app == "sssp" else 0
        ref = oracle.run_graph(app, g, 0, source=src)
        assert ref.status == oracle.OK
        for mode in ("auto", "push", "pull"):
            for persistent in (False, True):
                vals, st_ = dev.run(app, source=src, mode=mode, persistent=persistent)
                assert np.array_equal(ipg.values_to_numpy(vals), ref.values), (app, mode, persistent, store)
                assert np.array_equal(st_.trace, ref.trace), (app, mode, persistent, store)
    dev.close()
