"""Training data, GPU training and evaluation of the learned exchange selector.

Labels come from timing the plain method.  Every CC/SSSP run is repeated
with the exchange forced to each of the three variants the network scores --
a push that visits the frontier as a list, a push that sweeps every vertex's
mailbox, a pull -- in the configuration the selector is deployed with: a
store with the blocked in-edges, the device-driven superstep loop, and the
launch parameters the autotuner picks for that graph.  The state at the
start of a superstep does not depend on the exchange (values and traces are
identical in every run), so superstep s of the three runs starts from the
same state and their per-superstep device times (the decide kernel's
wall-clock stamps) give the three targets for that state: log2 of the
microseconds of each variant.  A list exists only after a push, so the
choices of a policy are replayed superstep by superstep with that
constraint when its time is summed.

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

    # Training graphs span the sizes of the workloads (up to ~270M edges: the
    # scale-23 symmetrised R-MAT stands in for the billion-edge one) with
    # seeds of their own; the held-out set includes the benchmark graphs
    # themselves (R-MAT s20 seed 2, the 4096^2 grid seed 3).
    if kind == "train":
        specs = [("rmat", 15, 11, True), ("rmat", 16, 12, True), ("rmat", 17, 13, False), ("rmat", 18, 14, True),
                 ("rmat", 19, 15, True), ("rmat", 18, 16, False), ("rmat", 21, 19, True), ("rmat", 20, 25, False),
                 ("rmat", 23, 26, True),
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


# The network's outputs, in order: (forced exchange, list_div) of each variant.
VARIANTS = (("push", 1), ("push", 0xFFFFFFFF), ("pull", None))
VARIANT_NAMES = ("push_list", "push_dense", "pull")


def time_runs(g, hg, name, runs, tun, reps, kind, verbose=True):
    """Per-superstep times of every variant for each (app, source) run:
    returns (T [steps,3] log2-usec, meta) pairs."""
    out = []
    for app, src in runs:
        times = []
        for mode, list_div in VARIANTS:
            t = dict(tun)
            if list_div is not None:
                t["list_div"] = list_div
            us = []
            for _ in range(reps):
                _, st = g.run(app, source=src, mode=mode, timing=True, tuning=t, persistent=True)
                us.append(st.usec.astype(np.float64))
            times.append(np.median(np.stack(us), axis=0))
        front = decision_frontier(app, st.active)
        T = np.log2(np.maximum(np.stack(times, axis=1), 1.0))
        meta = [(name, app, src, s, int(front[s]), int(st.frontier_deg[s]), int(hg.m), int(hg.n))
                for s in range(st.supersteps)]
        out.append((T, meta))
        if verbose:
            sums = ", ".join(f"{v} {np.exp2(T[:, i]).sum():.0f} us" for i, v in enumerate(VARIANT_NAMES))
            print(f"[selector] {kind} {name} {app} src={src} {tun}: {st.supersteps} supersteps, {sums}",
                  file=sys.stderr, flush=True)
    return out


def features(meta) -> np.ndarray:
    import paper_2010_08781_amd as ipg

    return ipg.selector_features([m[4] for m in meta], [m[5] for m in meta], [m[3] for m in meta],
                                 [m[6] for m in meta])


def collect(kind: str = "train", reps: int = 3, verbose: bool = True):
    """Returns (X [n,4], T [n,3] log2-usec per variant, meta list)."""
    import paper_2010_08781_amd as ipg

    from paper_2010_08781_amd import autotune

    T, meta = [], []
    for name, hg in _graphs(kind):
        g = ipg.Graph.from_host(hg, blocked=True)
        tun = autotune.tune(g, hg, "cc", cache_path=None, reps=1, persistent=True)
        for k in ("push_div", "list_div", "late_div"):  # the rule's divisors: irrelevant to forced variants
            tun.pop(k, None)
        runs = [("cc", 0)] + [("sssp", s) for s in _sources(hg, 4, 99)]
        for t, m in time_runs(g, hg, name, runs, tun, reps, kind, verbose):
            T.append(t)
            meta += m
        g.close()
    return features(meta), np.concatenate(T), meta


def init_params(seed: int = 1, scale: float = 0.5) -> np.ndarray:
    """Uniform(-scale/sqrt(fan_in), +scale/sqrt(fan_in)) weights, zero biases, packed as the library expects."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_out, fan_in in ((16, 4), (16, 16), (3, 16)):
        lim = scale / np.sqrt(fan_in)
        parts += [rng.uniform(-lim, lim, fan_out * fan_in), np.zeros(fan_out)]
    return np.concatenate(parts)


PUSH_LIST, PUSH_DENSE, PULL = 0, 1, 2


def replay(meta, pick) -> np.ndarray:
    """A policy's variant in every superstep: pick(i, list_available) for
    sample i, where a list is available only after a push (superstep 0's
    active set is given, so it has none)."""
    choice = np.empty(len(meta), dtype=np.int64)
    avail = False
    for i, m in enumerate(meta):
        if i == 0 or tuple(meta[i - 1][:3]) != tuple(m[:3]) or m[3] == 0:
            avail = False
        choice[i] = pick(i, avail)
        avail = choice[i] != PULL
    return choice


def heuristic_choice(meta, push_div: int = 20, list_div: int = 16) -> np.ndarray:
    """The fixed rule: pull when frontier + its out-degrees > E / push_div,
    else push over the list when there is one of at most max(4096, N / list_div)."""
    def pick(i, avail):
        _, _, _, _, f, d, e, n = meta[i]
        if e > 0 and f + d > e // push_div:
            return PULL
        return PUSH_LIST if avail and f <= max(4096, n // list_div) else PUSH_DENSE
    return replay(meta, pick)


def pick_from_outputs(y: np.ndarray, meta) -> np.ndarray:
    """The network's choice from its outputs y [n,3], as the library takes it."""
    def pick(i, avail):
        push = PUSH_LIST if avail and y[i, PUSH_LIST] <= y[i, PUSH_DENSE] else PUSH_DENSE
        return PULL if y[i, PULL] < y[i, push] else push
    return replay(meta, pick)


def regret(T: np.ndarray, choice: np.ndarray, meta=None) -> dict:
    """Time of the chosen variants against the fastest one in every
    superstep (the list variant counted only after superstep 0)."""
    t = np.exp2(T)  # microseconds
    chosen = t[np.arange(len(t)), choice]
    tb = t.copy()
    if meta is not None:
        tb[np.array([m[3] == 0 for m in meta], dtype=bool), PUSH_LIST] = np.inf
    best = tb.min(axis=1)
    return {"chosen_us": float(chosen.sum()), "best_us": float(best.sum()),
            "regret_us": float((chosen - best).sum()), "accuracy": float(np.mean(chosen <= best))}


def cost_weighted(X, T, cap: int = 16):
    """Replicate each sample in proportion to what a wrong choice costs there
    (the spread of the variants' times relative to the mean), so the
    squared-error fit is most accurate where the decision matters."""
    cost = np.exp2(T).max(axis=1) - np.exp2(T).min(axis=1)
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


def predict_choice(p, X, meta) -> np.ndarray:
    import torch

    import paper_2010_08781_amd as ipg

    y = ipg.selector_forward(p, torch.tensor(X, dtype=torch.float64, device="cuda")).cpu().numpy()
    return pick_from_outputs(y, meta)


def load(path: str = DEFAULT_PARAMS):
    """Trained parameters as a float64 CUDA tensor, or None if there are none."""
    import torch

    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    return torch.tensor(d["params"], dtype=torch.float64, device="cuda")


# Regret tables of the benchmark workloads: the runs the benchmark times, on
# the store it builds (blocked in-edges; cold sources binned, the 2^21
# hottest gathered, when the u32 value array fills the 256 MB Infinity
# Cache; weighted graphs pull by rows).
TABLE_RUNS = {"grid4096-sc": (("sssp", 0),), "rmat-s26-sym": (("cc", 0), ("sssp", 0)),
              "rmat-s20-sym": (("cc", 0), ("sssp", 0))}


def regret_table(workload: str, reps: int = 3) -> dict:
    """Per-superstep times of the three variants for the benchmark's runs
    on `workload`, with the raw inputs of both policies (the network's
    features and the fixed rule's frontier, out-degree sum, E and N)."""
    import torch

    import graphgen
    import paper_2010_08781_amd as ipg
    from paper_2010_08781_amd import autotune

    hg = graphgen.workload(workload)
    weighted = getattr(hg, "csr_w", None) is not None
    binned = not weighted and 4 * hg.n >= (256 << 20)
    hot = (1 << 21) if binned else 0
    g = ipg.Graph.from_host(hg, blocked=not weighted, binned=binned, binned_hot=hot)
    tun = autotune.tune(g, hg, TABLE_RUNS[workload][0][0], cache_path=None, reps=1, persistent=True)
    for k in ("push_div", "list_div", "late_div"):
        tun.pop(k, None)
    samples = []
    for T, meta in time_runs(g, hg, workload, TABLE_RUNS[workload], tun, reps, "table"):
        for t, m in zip(T, meta):
            samples.append({"app": m[1], "source": m[2], "superstep": m[3], "frontier": m[4], "frontier_deg": m[5],
                            "e": m[6], "n": m[7], "log2_us": [round(float(x), 6) for x in t]})
    g.close()
    return {"workload": workload, "graph": {"name": hg.name, "n": int(hg.n), "m": int(hg.m)},
            "store": {"blocked": not weighted, "binned": binned, "binned_hot": hot}, "tuning": tun, "reps": reps,
            "measured_on": torch.cuda.get_device_name(0), "when": time.strftime("%Y-%m-%d"),
            "variants": list(VARIANT_NAMES), "samples": samples}


def table_arrays(table: dict):
    """(T [n,3] log2-usec, meta) of a regret table."""
    meta = [(table["workload"], x["app"], x["source"], x["superstep"], x["frontier"], x["frontier_deg"], x["e"],
             x["n"]) for x in table["samples"]]
    return np.array([x["log2_us"] for x in table["samples"]], dtype=np.float64), meta


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_PARAMS)
    ap.add_argument("--epochs", type=int, default=30000)
    ap.add_argument("--lr", type=float, default=0.1)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--data-out", default=None, help="also write the timed samples (npz)")
    ap.add_argument("--data-in", default=None, help="train on samples written by --data-out instead of timing")
    ap.add_argument("--regret-table", default=None, choices=sorted(TABLE_RUNS),
                    help="only time the variants on this benchmark workload and write the table to --table-out")
    ap.add_argument("--table-out", default=None)
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(HERE))
    t0 = time.time()
    if args.regret_table:
        table = regret_table(args.regret_table, reps=args.reps)
        with open(args.table_out, "w") as f:
            json.dump(table, f, indent=0)
        print(f"[selector] wrote {args.table_out}: {len(table['samples'])} supersteps in {time.time() - t0:.0f}s",
              file=sys.stderr, flush=True)
        return
    if args.data_in:
        d = np.load(args.data_in, allow_pickle=False)

        def meta(m):
            return [(a, b, int(c), int(k), int(f), int(dd), int(e), int(n)) for a, b, c, k, f, dd, e, n in m]

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
        res[split] = {"samples": int(len(X)), "learned": regret(T, predict_choice(p, X, m), m),
                      "heuristic": regret(T, heuristic_choice(m), m),
                      "always_pull": regret(T, np.full(len(X), PULL), m),
                      "always_push": regret(T, replay(m, lambda i, a: PUSH_LIST if a else PUSH_DENSE), m)}
    out = {"params": pn.tolist(), "epochs": args.epochs, "lr": args.lr, "evaluation": res,
           "features": "log2(1+|F|)/32, log2(1+sum outdeg F)/32, min(s,128)/64, log2(1+E)/32",
           "targets": "log2 microseconds of a superstep exchanged by a push over the frontier list, a push "
                      "sweeping every vertex, a pull (device wall-clock stamps, median of reps)",
           "seconds": time.time() - t0}
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(res, indent=1))


if __name__ == "__main__":
    main()
