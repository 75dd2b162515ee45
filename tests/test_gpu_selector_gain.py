"""What the trained selector gains over the fixed rule, measured live on the
full 4096 x 4096 weighted grid with 1% shortcuts (SSSP from vertex 0, 92
supersteps), a graph the selector was not trained on.

Per-superstep times of the three variants the network scores (push over the
frontier list, push sweeping every vertex, pull) are taken in the
configuration the selector is deployed with (device-driven loop), with the
same superstep states in every run, since results and traces do not depend
on the exchange.  Both policies are then replayed over that one table (a
list exists only after a push), so the comparison itself has no timing
noise: the time the network's choices lose against the fastest variant must
not exceed the fixed rule's.
"""
import numpy as np
import pytest

import graphgen

pytestmark = pytest.mark.gpu


def test_trained_selector_regret_vs_rule_grid4096():
    import paper_2010_08781_amd as ipg
    from paper_2010_08781_amd import selector_fit as sf

    params = sf.load()
    assert params is not None, "selector_params.json missing"
    hg = graphgen.workload("grid4096-sc")
    g = ipg.Graph.from_host(hg)
    (T, meta), = sf.time_runs(g, hg, "grid4096-sc", [("sssp", 0)], {}, 3, "test")
    X = sf.features(meta)
    learned = sf.regret(T, sf.predict_choice(params, X, meta), meta)
    rule = sf.regret(T, sf.heuristic_choice(meta), meta)
    print(f"learned regret {learned['regret_us']:.0f} us, rule {rule['regret_us']:.0f} us, "
          f"best {rule['best_us']:.0f} us")
    assert learned["regret_us"] <= rule["regret_us"]
    # and the trained network drives a run to the same results as the rule
    a = ipg.values_to_numpy(g.run("sssp", source=0)[0])
    b = ipg.values_to_numpy(g.run("sssp", source=0, selector=params)[0])
    c = ipg.values_to_numpy(g.run("sssp", source=0, selector=params, persistent=True)[0])
    assert np.array_equal(a, b) and np.array_equal(a, c)
