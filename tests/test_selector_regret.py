"""The trained selector against the fixed rule on the benchmark workloads,
from committed timing tables (tests/data/selector_regret_*.json).

Each table holds, for every superstep of the benchmark's runs (the 4096 x
4096 weighted grid, SSSP from vertex 0; the symmetrised R-MAT scale 26, CC
and SSSP from vertex 0), the measured time of the three exchange variants
the network scores and the raw inputs of both policies.  They are timings of
the library on an MI355X (written by `selector_fit --regret-table`), inputs
of this comparison, not expected results of the method.  The committed
network (selector_params.json) is evaluated with the float64 reference MLP;
both policies are replayed over the table (a list exists only after a push),
and the time the network's choices lose against the fastest variant must not
exceed the fixed rule's (pull when frontier + out-degrees > E/20, list up to
max(4096, N/16)).
"""
import glob
import json
import os

import numpy as np
import pytest

from oracle import mlp
from paper_2010_08781_amd import selector_fit as sf
from paper_2010_08781_amd import selector_features

HERE = os.path.dirname(os.path.abspath(__file__))
TABLES = sorted(glob.glob(os.path.join(HERE, "data", "selector_regret_*.json")))


def test_tables_present():
    names = {os.path.basename(p) for p in TABLES}
    assert {"selector_regret_grid4096-sc.json", "selector_regret_rmat-s26-sym.json"} <= names


@pytest.mark.parametrize("path", TABLES, ids=[os.path.basename(p) for p in TABLES])
def test_learned_regret_not_above_rule(path):
    table = json.load(open(path))
    T, meta = sf.table_arrays(table)
    assert T.shape == (len(meta), 3) and np.isfinite(T).all()
    params = np.array(json.load(open(sf.DEFAULT_PARAMS))["params"], dtype=np.float64)
    assert params.size == mlp.n_params()
    X = selector_features([m[4] for m in meta], [m[5] for m in meta], [m[3] for m in meta], [m[6] for m in meta])
    y = mlp.forward(params, X)
    learned = sf.regret(T, sf.pick_from_outputs(y, meta), meta)
    rule = sf.regret(T, sf.heuristic_choice(meta), meta)
    print(f"{table['workload']}: learned regret {learned['regret_us']:.0f} us, rule {rule['regret_us']:.0f} us, "
          f"best {rule['best_us']:.0f} us")
    assert learned["regret_us"] <= rule["regret_us"]


def test_replay_keeps_lists_after_pushes_only():
    meta = [("w", "cc", 0, s, 10, 10, 1000, 100) for s in range(4)] + [("w", "sssp", 0, s, 10, 10, 1000, 100)
                                                                       for s in range(2)]
    seen = []
    sf.replay(meta, lambda i, avail: seen.append(avail) or (sf.PULL if i == 1 else sf.PUSH_DENSE))
    # superstep 0 of each run has no list; after the pull of sample 1 none either
    assert seen == [False, True, False, True, False, True]
