"""Writes the full-size expected results under tests/golden/ from the CPU
oracle and the seeded input generators only (nothing here touches the GPU
library).  The oracle's pull form under OpenMP (chunks of 1024 vertices dealt
round-robin, for balance on R-MAT's low-id hubs) is used for speed: its
output equals the sequential push form bit for bit, for any thread count and
chunk (tests/test_oracle_pull.py).

    python tests/golden/make_goldens.py [c5] [c3] [c4]

Files:
  rmat-s26.json  directed R-MAT scale 26 (seed 5): PageRank T = 10, d = 0.85,
                 sampled ranks, the rank sum and the trace; its symmetrised
                 form: hash-min CC and unit-weight SSSP from vertex 0, SHA-256
                 of the full u32 result, the trace and sampled values.
  grid4096.json  4096 x 4096 grid with 1 % shortcuts, weights in [1, 255]
                 (seed 3): weighted SSSP from vertex 0, as above.
  rmat-s22-batch.json  symmetrised R-MAT scale 22 (seed 4), 256 sources
                 (seed 40): SHA-256 of each query's distances, the summed
                 trace (the batched run's, a finished query adding zeros).
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import graphgen  # noqa: E402
import oracle  # noqa: E402

SAMPLES = 4096


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def sample_ids(g, seed: int) -> np.ndarray:
    """Seeded uniform ids plus the vertices with the largest in- and
    out-degree, vertex 0 and the last vertex, ascending and distinct."""
    rng = np.random.default_rng(seed)
    ids = set(rng.choice(g.n, size=min(SAMPLES, g.n), replace=False).tolist())
    ids.update(np.argsort(np.diff(g.csc_off))[-32:].tolist())
    ids.update(np.argsort(np.diff(g.csr_off))[-32:].tolist())
    ids.update([0, g.n - 1])
    return np.array(sorted(ids), dtype=np.int64)


def min_app(g, app, source, seed):
    t = time.time()
    r = oracle.run_pull(app, g, 0, source=source, threads=0, chunk=1024)
    assert r.status == oracle.OK, r.status
    ids = sample_ids(g, seed)
    print(f"[golden] {g.name} {app} src={source}: {r.supersteps} supersteps in {time.time() - t:.1f}s", flush=True)
    return {
        "source": int(source),
        "supersteps": int(r.supersteps),
        "sha256_u32": sha(r.values.astype(np.uint32)),
        "trace": r.trace.tolist(),
        "sample_ids": ids.tolist(),
        "sample_values": r.values[ids].astype(np.int64).tolist(),
        "reached": int(np.sum(r.values != oracle.INF)),
    }


def write(name, obj):
    path = os.path.join(HERE, name)
    with open(path, "w") as f:
        json.dump(obj, f, separators=(",", ":"))
        f.write("\n")
    print(f"[golden] wrote {path} ({os.path.getsize(path)} bytes)", flush=True)


def c5():
    t = time.time()
    d, s = graphgen.workload_pair("rmat-s26")
    print(f"[golden] rmat-s26: n={d.n} m={d.m} sym m={s.m} in {time.time() - t:.1f}s", flush=True)
    t = time.time()
    pr = oracle.run_pull("pagerank", d, 10, damping=0.85, threads=0, chunk=1024)
    assert pr.status == oracle.OK
    print(f"[golden] pagerank T=10 in {time.time() - t:.1f}s", flush=True)
    ids = sample_ids(d, 51)
    out = {
        "graph": {"name": d.name, "n": d.n, "m": d.m, "scale": 26, "edge_factor": 16, "seed": 5},
        "graph_sym": {"name": s.name, "n": s.n, "m": s.m},
        "pagerank": {
            "T": 10, "damping": 0.85, "supersteps": int(pr.supersteps), "trace": pr.trace.tolist(),
            "sample_ids": ids.tolist(), "sample_values_hex": [float(x).hex() for x in pr.values[ids]],
            "sum_hex": float(np.sum(pr.values, dtype=np.float64)).hex(),
        },
    }
    del pr
    out["cc"] = min_app(s, "cc", 0, 52)
    out["sssp"] = min_app(s, "sssp", 0, 53)
    write("rmat-s26.json", out)


def c3():
    t = time.time()
    g = graphgen.workload("grid4096-sc")
    print(f"[golden] {g.name}: n={g.n} m={g.m} in {time.time() - t:.1f}s", flush=True)
    out = {"graph": {"name": g.name, "n": g.n, "m": g.m, "width": 4096, "seed": 3},
           "sssp": min_app(g, "sssp", 0, 31)}
    write("grid4096.json", out)


def c4():
    g = graphgen.workload("rmat-s22-sym")
    src = graphgen.pick_sources(g, 256, seed=40)
    t = time.time()
    shas, steps = [], []
    total = np.zeros((0, 3), dtype=np.uint64)
    for q in src:
        r = oracle.run_pull("sssp", g, 0, source=int(q), threads=0, chunk=1024)
        assert r.status == oracle.OK
        shas.append(sha(r.values.astype(np.uint32)))
        steps.append(int(r.supersteps))
        if r.trace.shape[0] > total.shape[0]:
            total = np.vstack([total, np.zeros((r.trace.shape[0] - total.shape[0], 3), dtype=np.uint64)])
        total[: r.trace.shape[0]] += r.trace
    print(f"[golden] {g.name}: 256 queries in {time.time() - t:.1f}s", flush=True)
    write("rmat-s22-batch.json", {
        "graph": {"name": g.name, "n": g.n, "m": g.m, "scale": 22, "seed": 4},
        "sources": [int(x) for x in src], "source_seed": 40,
        "sha256_u32": shas, "supersteps": steps, "trace_sum": total.tolist(),
    })


if __name__ == "__main__":
    which = sys.argv[1:] or ["c3", "c4", "c5"]
    for w in which:
        {"c3": c3, "c4": c4, "c5": c5}[w]()
