"""What the trained selector gains over the fixed heuristic, measured live.

Per-superstep push and pull times are taken on a graph that was not used for
training, in the configuration the selector is deployed with (blocked
in-edges, device-driven loop), with the same superstep states in both runs,
since results and traces do not depend on the exchange; the time lost
against the faster exchange (regret) of the trained network must not exceed
the heuristic's, up to timing noise.
"""
import numpy as np
import pytest

import graphgen

pytestmark = pytest.mark.gpu


def test_trained_selector_regret_vs_heuristic():
    import paper_2010_08781_amd as ipg
    from paper_2010_08781_amd import selector_fit as st

    params = st.load()
    assert params is not None, "selector_params.json missing"
    hg = graphgen.rmat(19, 16, seed=21, symmetric=True)  # held out from training
    g = ipg.Graph.from_host(hg, blocked=True)
    X, T, meta = [], [], []
    for app, src in (("cc", 0), ("sssp", 0), ("sssp", 12345)):
        times = {}
        for mode in ("push", "pull"):
            us = [g.run(app, source=src, mode=mode, timing=True, persistent=True)[1].usec.astype(np.float64)
                  for _ in range(3)]
            times[mode] = np.median(np.stack(us), axis=0)
        _, s = g.run(app, source=src, mode="pull")
        front = st.decision_frontier(app, s.active)
        X.append(ipg.selector_features(front, s.frontier_deg, np.arange(s.supersteps), hg.m))
        T.append(np.log2(np.maximum(np.stack([times["push"], times["pull"]], axis=1), 1.0)))
        meta += [("g", app, src, k, int(front[k]), int(s.frontier_deg[k]), hg.m) for k in range(s.supersteps)]
    X, T = np.concatenate(X), np.concatenate(T)
    learned = st.regret(T, st.predict_choice(params, X))
    heur = st.regret(T, st.heuristic_choice(meta))
    print(f"learned regret {learned['regret_us']:.0f} us (acc {learned['accuracy']:.2f}), "
          f"heuristic {heur['regret_us']:.0f} us (acc {heur['accuracy']:.2f}), best {heur['best_us']:.0f} us")
    assert learned["regret_us"] <= 1.15 * heur["regret_us"] + 0.02 * heur["best_us"]
    # and the trained network drives a run to the same results as the heuristic
    a = ipg.values_to_numpy(g.run("sssp", source=0)[0])
    b = ipg.values_to_numpy(g.run("sssp", source=0, selector=params)[0])
    c = ipg.values_to_numpy(g.run("sssp", source=0, selector=params, persistent=True)[0])
    assert np.array_equal(a, b) and np.array_equal(a, c)
