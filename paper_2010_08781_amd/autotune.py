"""Autotuner of the exchange kernels' launch parameters.

For a graph and an application it times the runs of a small grid of
candidate parameter sets (ipg_tuning: the PageRank LDS outbox cache size,
the pull grid, the push/pull rule's divisor, the frontier-list limit, the
sender gate and the late push of CC/SSSP; on a graph with blocked in-edges
also the row-item form of the pull) and keeps the fastest.  The choice is cached in a JSON file under a key made of
the graph's signature -- vertex and edge counts, symmetry, weights, naming
and a coarse profile of its out-degrees -- so a graph of the same shape is
not tuned twice.  Parameters never change results beyond the PageRank
summation-order freedom, so tuning needs no correctness check of its own.

    from paper_2010_08781_amd import autotune
    best = autotune.tune(graph, hg, "pagerank")       # dict for Graph.run(tuning=...)
"""
from __future__ import annotations

import hashlib
import itertools
import json
import os
import time
from typing import Optional

import numpy as np

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "ipregel_tuning.json")

# Candidate values per application (0 = the library's default).
SPACES = {
    "pagerank": {"pr_hot": [0xFFFFFFFF, 2048, 4096, 8192, 11200], "pull_grid": [1024, 2048, 4096]},
    "cc": {"push_div": [10, 20, 40], "list_div": [8, 16, 32], "pull_grid": [2048, 4096], "gate_div": [4, 16]},
    "sssp": {"push_div": [10, 20, 40], "list_div": [8, 16, 32], "pull_grid": [2048, 4096], "gate_div": [4, 16]},
    "multi_sssp": {"push_div": [5, 10, 20, 40], "pull_grid": [1024, 2048, 4096]},
}


def signature(hg, graph) -> str:
    """Key of a graph's shape: sizes, flags and the out-degree histogram in
    powers of two (rounded to 1% of the vertices)."""
    deg = np.diff(np.asarray(hg.csr_off, dtype=np.int64))
    hist = np.bincount(np.floor(np.log2(deg + 1)).astype(np.int64), minlength=32)
    hist = np.round(hist / max(hg.n, 1) * 100).astype(int).tolist()
    desc = {"n": int(hg.n), "m": int(len(hg.csr_dst)), "sym": bool(getattr(hg, "symmetric", False)),
            "w": getattr(hg, "csr_w", None) is not None, "renamed": bool(getattr(graph, "renamed", False)),
            "deg": hist}
    if getattr(graph, "blocked", False):
        desc["blocked"] = True
    return hashlib.sha1(json.dumps(desc, sort_keys=True).encode()).hexdigest()[:16]


def _load(path):
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def _save(path, cache):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def candidates(graph, app: str) -> list:
    """The parameter sets tried for `app` on this graph: the product of the
    application's space; on a graph with blocked in-edges also the blocked
    pull (PageRank: no launch parameters; CC/SSSP: the exchange rule's
    divisors, with and without the sender gate) before the row-item pull
    over the space."""
    space = SPACES[app]
    names = sorted(space)
    out = [dict(zip(names, combo)) for combo in itertools.product(*(space[k] for k in names))]
    # CC/SSSP: the late push at its default divisor and switched off
    late = (0, 0xFFFFFFFF) if app in ("cc", "sssp") else ()
    if getattr(graph, "blocked", False):
        if app == "pagerank":
            out = [{"blocked": 0}] + [dict(t, blocked=0xFFFFFFFF) for t in out]
        elif app in ("cc", "sssp"):
            # the blocked pull has no grid; the rule's divisors, the sender gate and the late push still matter
            blk = [dict(zip(("list_div", "push_div", "gate_div", "late_div"), c), blocked=0)
                   for c in itertools.product(space["list_div"], space["push_div"], (0, 0xFFFFFFFF), late)]
            out = blk + [dict(t, blocked=0xFFFFFFFF) for t in out]
    elif late:
        out = [dict(t, late_div=x) for t in out for x in late]
    return out


def _runner(graph, app, kw):
    if app == "pagerank":
        return lambda t: graph.run("pagerank", kw.get("updates", 10), mode="pull", tuning=t, timing=False)[1]
    if app in ("cc", "sssp"):
        return lambda t: graph.run(app, source=kw.get("source", 0), tuning=t, timing=False,
                                   persistent=kw.get("persistent", False))[1]
    if app == "multi_sssp":
        out = kw.get("out")
        return lambda t: graph.run_multi_sssp(kw["sources"], tuning=t, timing=False, out=out)[1]
    raise KeyError(app)


def tune(graph, hg, app: str, cache_path: Optional[str] = DEFAULT_CACHE, reps: int = 3, retune: bool = False,
         verbose: bool = False, **kw) -> dict:
    """Best parameter set for `app` on this graph (from the cache when the
    graph's signature was tuned before).  Extra keywords go to the runs:
    updates (PageRank), source / persistent (CC, SSSP), sources (multi_sssp)."""
    key = f"{app}:{signature(hg, graph)}"
    cache = _load(cache_path)
    if not retune and key in cache:
        return dict(cache[key]["tuning"])
    run = _runner(graph, app, kw)
    results = []
    run(None)  # warm-up (first-touch of the workspaces)
    for t in candidates(graph, app):
        run(t)
        secs = [run(t).seconds for _ in range(reps)]
        results.append((float(np.median(secs)), t))
        if verbose:
            print(f"[autotune] {app} {t}: {np.median(secs) * 1e3:.3f} ms", flush=True)
    default = float(np.median([run(None).seconds for _ in range(reps)]))
    best_s, best = min(results, key=lambda r: r[0])
    if cache_path:
        cache[key] = {"tuning": best, "ms": best_s * 1e3, "default_ms": default * 1e3, "candidates": len(results),
                      "when": time.strftime("%Y-%m-%d %H:%M:%S")}
        _save(cache_path, cache)
    return dict(best)


def report(cache_path: Optional[str] = DEFAULT_CACHE) -> dict:
    """The cached choices with their times against the defaults."""
    return _load(cache_path)
