"""Host logic of the autotuner: graph signatures and the tuning cache
(a stand-in graph object supplies run times; no GPU needed)."""
import json
from types import SimpleNamespace

import numpy as np

import graphgen
from paper_2010_08781_amd import autotune
from tests.graphs_small import random_graph


def test_signature_depends_on_shape_only():
    a = graphgen.rmat(10, 8, seed=1)
    b = graphgen.rmat(10, 8, seed=1)
    c = graphgen.rmat(10, 8, seed=2, symmetric=True)
    g = SimpleNamespace(renamed=True)
    assert autotune.signature(a, g) == autotune.signature(b, g)
    assert autotune.signature(a, g) != autotune.signature(c, g)
    assert autotune.signature(a, g) != autotune.signature(a, SimpleNamespace(renamed=False))


class FakeGraph:
    """run() takes longer the further pr_hot is from 4096 and pull_grid from 2048."""

    renamed = True

    def __init__(self):
        self.calls = 0

    def run(self, app, *a, tuning=None, **kw):
        self.calls += 1
        t = tuning or {}
        cost = 1.0 + abs(t.get("pr_hot", 8192) - 4096) / 1e4 + abs(t.get("pull_grid", 2048) - 2048) / 1e4
        return None, SimpleNamespace(seconds=cost * 1e-3)


def test_tune_picks_the_fastest_and_caches(tmp_path):
    hg = random_graph(200, 800, seed=1)
    g = FakeGraph()
    path = str(tmp_path / "cache.json")
    best = autotune.tune(g, hg, "pagerank", cache_path=path, reps=2)
    assert best == {"pr_hot": 4096, "pull_grid": 2048}
    calls = g.calls
    assert autotune.tune(g, hg, "pagerank", cache_path=path) == best and g.calls == calls  # from the cache
    entry = json.load(open(path))[f"pagerank:{autotune.signature(hg, g)}"]
    assert entry["candidates"] == 15 and entry["ms"] <= entry["default_ms"]
    autotune.tune(g, hg, "pagerank", cache_path=path, retune=True)
    assert g.calls > calls
