"""Training data, GPU training and evaluation of the learned exchange selector.

Labels come from timing the plain method.  Every CC/SSSP run is repeated
with the exchange forced to push and forced to pull, in the configuration
the selector is deployed with: a store with the blocked in-edges, the
device-driven superstep loop, and the launch parameters the autotuner picks
for that graph.  The state at the start of a superstep does not depend on
the exchange (values and traces are identical in both runs), so superstep s
of the two runs starts from the same state and their per-superstep device
times (the decide kernel's wall-clock stamps) give the two targets for that
state: log2 of the microseconds of a push and of a pull superstep.

The network is then trained on the device by the library's own FP64 forward,
backward and SGD kernels (ipg_selector_train), and compared with the fixed
heuristic on held-out graphs by its regret: the time lost against choosing
the faster exchange in every superstep.

    python -m paper_2010_08781_amd.selector_fit --out paper_2010_08781_amd/selector_params.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_PARAMS = os.path.join(HERE, "selector_params.json")


def _graphs(kind: str):
    import graphgen

    # Training graphs span the sizes of the workloads (up to ~67M edges) with
    # seeds of their own; the held-out set includes the benchmark graphs
    # themselves (R-MAT s20 seed 2, the 4096^2 grid seed 3).
    if kind == "train":
        specs = [("rmat", 15, 11, True), ("rmat", 16, 12, True), ("rmat", 17, 13, False), ("rmat", 18, 14, True),
                 ("rmat", 19, 15, True), ("rmat", 18, 16, False), ("rmat", 21, 19, True), ("rmat", 20, 25, False),
                 ("grid", 512, 17, None), ("grid", 1024, 18, None), ("grid", 2048, 20, None), ("grid", 4096, 24, None)]
    else:
        specs = [("rmat", 19, 21, True), ("rmat", 17, 22, False), ("grid", 768, 23, None), ("rmat", 20, 2, True),
                 ("grid", 4096, 3, None)]
    for s in specs:
        if s[0] == "rmat":
            yield f"rmat-s{s[1]}-{'sym' if s[3] else 'dir'}-seed{s[2]}", graphgen.rmat(s[1], 16, seed=s[2], symmetric=s[3])
        else:
            yield f"grid{s[1]}-seed{s[2]}", graphgen.grid_with_shortcuts(s[1], 0.01, seed=s[2])


def _sources(hg, k, seed):
    import graphgen

    return [0] + [int(x) for x in graphgen.pick_sources(hg, k, seed)]


def decision_frontier(app: str, active) -> np.ndarray:
    """Vertices whose messages the exchange of each superstep sends, as the
    decision sees them: the trace's active counts, except at superstep 0,
    where every vertex is active but only CC's all send (SSSP: the source)."""
    f = np.asarray(active, dtype=np.uint64).copy()
    if app == "sssp" and f.size:
        f[0] = 1
    return f


def collect(kind: str = "train", reps: int = 3, verbose: bool = True):
    """Returns (X [n,4], T [n,2] log2-usec for push/pull, meta list)."""
    import paper_2010_08781_amd as ipg

    from paper_2010_08781_amd import autotune

    X, T, meta = [], [], []
    for name, hg in _graphs(kind):
        g = ipg.Graph.from_host(hg, blocked=True)
        tun = autotune.tune(g, hg, "cc", cache_path=None, reps=1, persistent=True)
        tun.pop("push_div", None)  # the fixed rule's divisor: irrelevant to forced exchanges
        runs = [("cc", 0)] + [("sssp", s) for s in _sources(hg, 4, 99)]
        for app, src in runs:
            times = {}
            for mode in ("push", "pull"):
                us = []
                for _ in range(reps):
                    _, st = g.run(app, source=src, mode=mode, timing=True, tuning=tun, persistent=True)
                    us.append(st.usec.astype(np.float64))
                times[mode] = np.median(np.stack(us), axis=0)
            front = decision_frontier(app, st.active)
            feats = ipg.selector_features(front, st.frontier_deg, np.arange(st.supersteps), hg.m)
            X.append(feats)
            T.append(np.log2(np.maximum(np.stack([times["push"], times["pull"]], axis=1), 1.0)))
            meta += [(name, app, src, s, int(front[s]), int(st.frontier_deg[s]), hg.m) for s in range(st.supersteps)]
            if verbose:
                print(f"[selector] {kind} {name} {app} src={src} {tun}: {st.supersteps} supersteps, "
                      f"push {times['push'].sum():.0f} us, pull {times['pull'].sum():.0f} us", file=sys.stderr, flush=True)
        g.close()
    return np.concatenate(X), np.concatenate(T), meta


def init_params(seed: int = 1, scale: float = 0.5) -> np.ndarray:
    """Uniform(-scale/sqrt(fan_in), +scale/sqrt(fan_in)) weights, zero biases, packed as the library expects."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_out, fan_in in ((16, 4), (16, 16), (2, 16)):
        lim = scale / np.sqrt(fan_in)
        parts += [rng.uniform(-lim, lim, fan_out * fan_in), np.zeros(fan_out)]
    return np.concatenate(parts)


def heuristic_choice(meta) -> np.ndarray:
    """1 = pull, 0 = push, by the fixed rule (frontier + its out-degrees > E/20)."""
    return np.array([1 if (e > 0 and f + d > e // 20) else 0 for (_, _, _, _, f, d, e) in meta])


def regret(T: np.ndarray, choice: np.ndarray) -> dict:
    t = np.exp2(T)  # microseconds
    chosen = t[np.arange(len(t)), choice]
    best = t.min(axis=1)
    return {"chosen_us": float(chosen.sum()), "best_us": float(best.sum()),
            "regret_us": float((chosen - best).sum()), "accuracy": float(np.mean(chosen == best))}


def cost_weighted(X, T, cap: int = 16):
    """Replicate each sample in proportion to what a wrong choice costs there
    (|t_push - t_pull| relative to the mean), so the squared-error fit is
    most accurate where the decision matters."""
    cost = np.abs(np.exp2(T[:, 0]) - np.exp2(T[:, 1]))
    reps = 1 + np.minimum(np.floor(4.0 * cost / max(cost.mean(), 1e-9)), cap - 1).astype(np.int64)
    return np.repeat(X, reps, axis=0), np.repeat(T, reps, axis=0)


def train(X, T, epochs: int = 30000, lr: float = 0.1, seed: int = 1, weighted: bool = False):
    """Full-batch gradient descent on the library's kernels.  The squared
    error of the log-times is already relative, so the samples are used as
    they are; cost replication (weighted=True) fitted the rare, costly dense
    supersteps at the expense of the decisions near the crossover."""
    import torch

    import paper_2010_08781_amd as ipg

    if weighted:
        X, T = cost_weighted(X, T)
    p = torch.tensor(init_params(seed), dtype=torch.float64, device="cuda")
    x = torch.tensor(X, dtype=torch.float64, device="cuda")
    t = torch.tensor(T, dtype=torch.float64, device="cuda")
    ipg.selector_train(p, x, t, epochs=epochs, lr=lr)
    torch.cuda.synchronize()
    return p


def predict_choice(p, X) -> np.ndarray:
    import torch

    import paper_2010_08781_amd as ipg

    y = ipg.selector_forward(p, torch.tensor(X, dtype=torch.float64, device="cuda")).cpu().numpy()
    return (y[:, 1] < y[:, 0]).astype(np.int64)


def load(path: str = DEFAULT_PARAMS):
    """Trained parameters as a float64 CUDA tensor, or None if there are none."""
    import torch

    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    return torch.tensor(d["params"], dtype=torch.float64, device="cuda")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_PARAMS)
    ap.add_argument("--epochs", type=int, default=30000)
    ap.add_argument("--lr", type=float, default=0.1)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--data-out", default=None, help="also write the timed samples (npz)")
    ap.add_argument("--data-in", default=None, help="train on samples written by --data-out instead of timing")
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(HERE))
    t0 = time.time()
    if args.data_in:
        d = np.load(args.data_in, allow_pickle=False)

        def meta(m):
            return [(a, b, int(c), int(k), int(f), int(dd), int(e)) for a, b, c, k, f, dd, e in m]

        Xtr, Ttr, mtr, Xte, Tte, mte = d["Xtr"], d["Ttr"], meta(d["mtr"]), d["Xte"], d["Tte"], meta(d["mte"])
    else:
        Xtr, Ttr, mtr = collect("train", reps=args.reps)
        Xte, Tte, mte = collect("test", reps=args.reps)
    if args.data_out:
        np.savez(args.data_out, Xtr=Xtr, Ttr=Ttr, mtr=np.array(mtr, dtype=object).astype(str), Xte=Xte, Tte=Tte,
                 mte=np.array(mte, dtype=object).astype(str))
    p = train(Xtr, Ttr, epochs=args.epochs, lr=args.lr)
    pn = p.cpu().numpy()
    res = {}
    for split, X, T, m in (("train", Xtr, Ttr, mtr), ("heldout", Xte, Tte, mte)):
        res[split] = {"samples": int(len(X)), "learned": regret(T, predict_choice(p, X)),
                      "heuristic": regret(T, heuristic_choice(m)),
                      "always_pull": regret(T, np.ones(len(X), dtype=np.int64)),
                      "always_push": regret(T, np.zeros(len(X), dtype=np.int64))}
    out = {"params": pn.tolist(), "epochs": args.epochs, "lr": args.lr, "evaluation": res,
           "features": "log2(1+|F|)/32, log2(1+sum outdeg F)/32, min(s,128)/64, log2(1+E)/32",
           "targets": "log2 microseconds of a push and of a pull superstep (HIP events, median of reps)",
           "seconds": time.time() - t0}
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(res, indent=1))


if __name__ == "__main__":
    main()
