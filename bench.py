#!/usr/bin/env python3
"""Benchmark of the superstep engine on one MI355X.

One step = one pass of the whole hot path over the workload: PageRank (10
rank updates, d = 0.85, FP64, pull exchange) on the directed graph, then
hash-min connected components and SSSP from vertex 0, each to vote-to-halt,
on its symmetrised form (push/pull chosen per superstep by the trained
selector, device-driven superstep loop), with launch parameters from the
autotuner.  Default workload: the billion-edge configuration, synthetic
R-MAT scale 26, edge factor 16, seed 5 (67.1M vertices; 1.06B directed
edges, 2.10B symmetrised).  Graphs are resident in HBM before timing starts.
A shorter pass of the same step on R-MAT scale 20 symmetrised (seed 2) is
reported as a secondary object.

Prints ONE JSON line.  `value` = GTEPS over the step: messages delivered
(edges traversed by the method: the senders' out-degrees, summed over
supersteps and applications) / step wall time.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GTEPS/superstep + time-to-converge (PR/CC/SSSP), learned+batched vs plain"
HBM_PEAK_GBS = 8000.0


def pr_pull_bytes(n: int, m: int) -> int:
    """Algorithmic HBM bytes of one PageRank pull superstep: CSC sources (4 B
    per edge), CSC offsets (8 B per vertex + 1), the outbox read once (8 B per
    vertex), the out-degree (4 B) and the new outbox or rank (8 B)."""
    return 4 * m + 8 * (n + 1) + 8 * n + 4 * n + 8 * n


# HBM traffic of the PageRank pull kernel from the committed rocprofv3 PMC
# summary: valid only while the kernel sources are the ones it was taken on.
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "pr_pull_traffic_{workload}.md")
KERNEL_SOURCES = ("paper_2010_08781_amd/csrc/pagerank.hip", "paper_2010_08781_amd/csrc/common.h",
                  "paper_2010_08781_amd/csrc/blocked_layout.h", "paper_2010_08781_amd/csrc/blocked.h",
                  "paper_2010_08781_amd/csrc/engine.h", "paper_2010_08781_amd/csrc/store.hip")


def kernel_source_hash() -> str:
    import hashlib

    h = hashlib.sha1()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:12]


def measured_traffic(workload: str, tuning) -> "int | None":
    """Bytes per superstep (FETCH_SIZE + WRITE_SIZE, each scaled by the copy
    calibration) recorded for this workload and launch parameters, or None."""
    import re

    path = TRAFFIC_SUMMARY.format(workload=workload)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"traffic_bytes_per_superstep:\s*(\d+)\s+sources:\s*([0-9a-f]+)\s+tuning:\s*(\{.*\})", text)
    if not m or m.group(2) != kernel_source_hash():
        return None
    if json.loads(m.group(3)) != (tuning or {}):
        return None
    return int(m.group(1))


def batched_vs_plain(ipg, graphgen, np, torch, reps: int = 3, tune_cache=None, cap: int = 64) -> dict:
    """End-to-end time of the batched workload against the plain form on the
    same GPU: 256 unit-weight SSSP queries (sources seeded among vertices with
    out-edges) on R-MAT scale 22 symmetrised, plus 64 directed R-MAT graphs
    (2^10..2^16 vertices, edge factor 8) with 20 PageRank updates each.
    Batched = one hipGraph launch holding the device-driven batched SSSP
    (supersteps enqueued up to a fixed cap, not sized from this batch) and
    the PageRank run over the union with per-part N; plain = 256
    single-source runs in the library's best single-source form (device-driven
    loop, autotuned launch parameters, the fixed rule's exchange) + 64
    separate PageRank runs, each replayed as one hipGraph.  Inputs resident
    before timing."""
    from paper_2010_08781_amd import autotune
    from paper_2010_08781_amd.batch import BatchPlan

    hg = graphgen.workload("rmat-s22-sym")
    src = graphgen.pick_sources(hg, 256, seed=40)
    g = ipg.Graph.from_host(hg)
    fam = graphgen.small_graph_family(64, seed=41)
    u = graphgen.disjoint_union(fam, name="family64")
    gu = ipg.Graph.from_host(u)
    parts = torch.from_numpy(u.meta["parts"].astype(np.int32)).cuda()
    gs = [ipg.Graph.from_host(h) for h in fam]
    d = torch.empty((256, g.n), dtype=torch.int32, device="cuda")

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        return float(np.median(ts))

    tms = autotune.tune(g, hg, "multi_sssp", cache_path=tune_cache, reps=1, sources=src, out=d) if tune_cache else None
    tpr = autotune.tune(gu, u, "pagerank", cache_path=tune_cache, reps=1, updates=20) if tune_cache else None
    # the plain single-source form at its best: launch parameters tuned for SSSP on this graph
    tss = autotune.tune(g, hg, "sssp", cache_path=tune_cache, reps=1, persistent=True) if tune_cache else None
    plan = BatchPlan(g, src, gu, parts, updates=20, max_supersteps=cap, sssp_tuning=tms, pr_tuning=tpr).capture()

    def one_launch():
        plan.replay()

    def b_sssp():
        g.run_multi_sssp(src, out=d, persistent=True, timing=False, tuning=tms)

    def p_sssp():
        for s in src:
            g.run("sssp", source=int(s), timing=False, persistent=True, tuning=tss)

    def b_pr():
        gu.run("pagerank", 20, mode="pull", parts=parts, graph=True, timing=False, tuning=tpr)

    def p_pr():
        for h in gs:
            h.run("pagerank", 20, mode="pull", timing=False, graph=True)

    t = {"one": timed(one_launch), "b_sssp": timed(b_sssp), "p_sssp": timed(p_sssp), "b_pr": timed(b_pr),
         "p_pr": timed(p_pr)}
    st = plan.sssp()[1]
    assert st.status == ipg.OK and st.supersteps < cap
    # every query of the replayed plan equals the library's own single-source run
    dist = plan.sssp()[0].cpu().numpy()
    for i, s in enumerate(src):
        one, _ = g.run("sssp", source=int(s), timing=False, persistent=True, tuning=tss)
        assert np.array_equal(one.cpu().numpy(), dist[i]), f"batched query {i} differs from its single-source run"
    out = {"sssp256_rmat_s22": {"batched_ms": round(t["b_sssp"] * 1e3, 3), "plain_ms": round(t["p_sssp"] * 1e3, 3),
                                "speedup": round(t["p_sssp"] / t["b_sssp"], 2), "supersteps": st.supersteps,
                                "edges_traversed": st.edges_traversed, "tuning": tms, "plain_tuning": tss,
                                "plain_form": "device-driven single-source runs, autotuned, fixed rule",
                                "plan_superstep_cap": cap, "queries_checked_against_single_source": 256},
           "pagerank64_family": {"batched_ms": round(t["b_pr"] * 1e3, 3), "plain_ms": round(t["p_pr"] * 1e3, 3),
                                 "speedup": round(t["p_pr"] / t["b_pr"], 2), "n": u.n, "m": u.m, "tuning": tpr}}
    tp = t["p_sssp"] + t["p_pr"]
    out["end_to_end"] = {"batched_ms": round(t["one"] * 1e3, 3), "plain_ms": round(tp * 1e3, 3),
                         "speedup": round(tp / t["one"], 2),
                         "form": f"one hipGraph launch (batched SSSP up to {cap} supersteps + PageRank union)"}
    for h in gs + [g, gu]:
        h.close()
    return out


def host_info() -> dict:
    """Cores, CPU model and memory of the host the oracle baseline runs on."""
    info = {"nproc": os.cpu_count()}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    info["cpu_model"] = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    info["ram_gib"] = round(int(line.split()[1]) / 2**20, 1)
                    break
    except OSError:
        pass
    return info


def load_workload(name: str):
    """(graph for PageRank, graph for CC/SSSP): the directed and symmetrised
    forms of one R-MAT draw for "rmat-s26", else one graph for both."""
    import graphgen

    if name == "rmat-s26":
        return graphgen.workload_pair("rmat-s26")
    hg = graphgen.workload(name)
    return hg, hg


def bench_workload(name, args, sel, ipg, np, torch, steps, warmup, apps, tune_cache):
    """Builds the workload's device graphs, tunes, then times `steps` steps
    after `warmup`; returns the measurements of one workload."""
    t0 = time.perf_counter()
    h_pr, h_min = load_workload(name)
    print(f"[bench] generated {name}: n={h_pr.n} m={h_pr.m}"
          f"{'' if h_min is h_pr else f' (symmetrised m={h_min.m})'} in {time.perf_counter() - t0:.1f}s",
          file=sys.stderr, flush=True)
    T = args.pr_updates
    graphs = {}
    t0 = time.perf_counter()
    # binned cold sources when the vertex-value array (8 bytes per vertex for
    # PageRank, 4 for the minima) fills the 256 MB Infinity Cache
    def binned(n, width):
        return not args.no_blocked and (args.binned == "on" or (args.binned == "auto" and width * n >= (256 << 20)))

    if "pagerank" in apps:
        graphs["pagerank"] = ipg.Graph.from_host(h_pr, blocked=not args.no_blocked, binned=binned(h_pr.n, 8),
                                                 binned_hot=args.binned_hot)
        print(f"[bench] PageRank graph created in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    if any(a != "pagerank" for a in apps):
        # the hot sources' values held in 8 MB either way: 2^20 FP64 outboxes
        # for PageRank (the library's default), 2^21 u32 ones for CC/SSSP
        gm = graphs["pagerank"] if h_min is h_pr and "pagerank" in graphs else \
            ipg.Graph.from_host(h_min, blocked=not args.no_blocked, binned=binned(h_min.n, 4),
                                binned_hot=args.binned_hot or (1 << 21))
        for a in apps:
            if a != "pagerank":
                graphs[a] = gm
    host = {a: (h_pr if a == "pagerank" else h_min) for a in apps}
    print(f"[bench] device graphs created in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)

    def run(app, selector=sel, tuning=None, source=0, timing=True):
        if app == "pagerank":
            return graphs[app].run("pagerank", T, mode="pull", timing=timing, tuning=tuning)
        return graphs[app].run(app, source=source, mode=args.mode, timing=timing, selector=selector, tuning=tuning,
                               persistent=True)

    # cold: the first device-driven run of each application on the fresh
    # handle (one-time per-handle setup included, first chunk of 2 supersteps)
    cold = {}
    for app in apps:
        if app != "pagerank":
            t = time.perf_counter()
            _, st = run(app)
            cold[app] = {"time_to_converge_ms": round(st.seconds * 1e3, 4),
                         "wall_ms": round((time.perf_counter() - t) * 1e3, 4)}

    tun = {app: None for app in apps}
    if not args.no_tune:
        from paper_2010_08781_amd import autotune

        t0 = time.perf_counter()
        for app in apps:
            tun[app] = autotune.tune(graphs[app], host[app], app, cache_path=tune_cache, reps=2, updates=T,
                                     persistent=True)
        print(f"[bench] {name}: autotuned {tun} in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)

    def one_step(selector=sel):
        return {app: run(app, selector, tun[app])[1] for app in apps}

    for i in range(warmup):
        one_step()
        print(f"[bench] {name}: warmup {i + 1}/{warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    per_step = [one_step() for _ in range(steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    edges_per_step = sum(st.edges_traversed for st in per_step[0].values())

    apps_out = {}
    for app in apps:
        sts = [s[app] for s in per_step]
        secs = np.array([s.seconds for s in sts])
        st = sts[0]
        apps_out[app] = {
            "graph": host[app].name, "n": host[app].n, "m": host[app].m,
            "supersteps": st.supersteps,
            "edges_traversed": st.edges_traversed,
            "edges_examined": st.edges_examined,
            "time_to_converge_ms_median": float(np.median(secs) * 1e3),
            "gteps": float(st.edges_traversed / np.median(secs) / 1e9),
            "us_per_superstep": float(np.median(secs) * 1e6 / st.supersteps),
            "modes": "".join("?PL"[int(x)] for x in st.mode),
        }
        if app in cold:
            apps_out[app]["cold"] = cold[app]

    # SSSP from rotating sources: each run's first chunk is sized by the
    # previous run, from another source
    if "sssp" in apps:
        import graphgen

        srcs = graphgen.pick_sources(host["sssp"], 8, seed=7)
        secs = [run("sssp", source=int(v), tuning=tun["sssp"])[1].seconds for v in srcs]
        apps_out["sssp"]["rotating_sources_ms_median"] = round(float(np.median(secs)) * 1e3, 4)

    # The same CC/SSSP runs (outside the timed region) with the exchange
    # picked by the fixed rule instead of the trained network: at the rule's
    # documented divisors (pull when frontier + out-edges > E/20, lists up to
    # N/16: the plain method) and at the divisors the autotuner picked;
    # other launch parameters as tuned.
    learned_vs_plain = None
    if sel is not None:
        learned_vs_plain = {}
        for app in apps:
            if app == "pagerank":
                continue
            t_plain = dict(tun[app] or {})
            t_plain["push_div"] = 20
            t_plain["list_div"] = 16

            def med(t):
                return float(np.median([run(app, selector=None, tuning=t)[1].seconds for _ in range(max(3, steps))]))

            plain, rule = med(t_plain), med(tun[app])
            mine = apps_out[app]["time_to_converge_ms_median"] / 1e3
            learned_vs_plain[app] = {"learned_ms": round(mine * 1e3, 4), "plain_ms": round(plain * 1e3, 4),
                                     "speedup": round(plain / mine, 4),
                                     "tuned_rule_ms": round(rule * 1e3, 4), "speedup_vs_tuned_rule": round(rule / mine, 4),
                                     "learned_beats_tuned_rule": bool(mine < rule),
                                     "note": (f"the trained network is {rule / mine:.3f}x the autotuned rule: "
                                              + ("not faster" if mine >= rule else "faster")
                                              + f"; {plain / mine:.3f}x the plain E/20 rule")}

    roofline = None
    if "pagerank" in apps and T >= 1:
        # average duration of one pull superstep from HIP events recorded on
        # the launch stream around each superstep
        us = np.concatenate([s["pagerank"].usec[1:T + 1] for s in per_step])
        avg_us = float(np.mean(us))
        nbytes = pr_pull_bytes(h_pr.n, h_pr.m)
        ach = nbytes / (avg_us * 1e-6) / 1e9
        g = graphs["pagerank"]
        traffic = measured_traffic(h_pr_key(name), tun.get("pagerank"))
        blocked = g.blocked and (tun.get("pagerank") or {}).get("blocked", 0) != 0xFFFFFFFF
        kernel = (("pr_bin_kernel + " if blocked and g.binned else "") +
                  ("pr_blocked_kernel + pr_blocked_finish_kernel" if blocked else
                   "pr_items_kernel + pr_longrow_kernel") + " (one PageRank pull superstep)")
        roofline = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "kernel": kernel, "graph": h_pr.name,
                    "bytes_per_launch": nbytes, "bytes_formula": "4E + 8(N+1) + 8N + 4N + 8N",
                    "avg_launch_us": round(avg_us, 2),
                    "tuning": tun.get("pagerank"), "kernel_sources": kernel_source_hash()}

    out = {"name": name, "steps": steps, "warmup": warmup, "wall_s": wall,
           "ms_per_step": wall / steps * 1e3, "value": edges_per_step * steps / wall / 1e9,
           "apps": apps_out, "tuning": tun, "learned_vs_plain": learned_vs_plain, "roofline": roofline,
           "host": host, "graphs": graphs}
    return out


def h_pr_key(name: str) -> str:
    """Name of the committed traffic summary of the workload's PageRank graph."""
    return "rmat-s26-dir" if name == "rmat-s26" else name


def cpu_baseline(name, host, apps, T, np) -> dict:
    """The oracle timed on the host's cores: its pull form with the vertex loop
    under OpenMP's default static schedule (the paper's parallelisation), on
    a bounded sample of the workload -- at scale 26 the first rank update of
    PageRank (supersteps 0-1) and the first two supersteps of CC and SSSP."""
    import oracle

    threads = oracle.max_threads()
    big = host[apps[0]].m > 100_000_000
    secs, msgs, parts = 0.0, 0, []
    for app in apps:
        hg = host[app]
        if app == "pagerank":
            param = 1 if big else T
        else:
            param = 2 if big else 0
        r = oracle.run_pull(app, hg, param, source=0, threads=threads)
        assert r.status in (oracle.OK, oracle.NOT_CONVERGED)
        secs += r.seconds
        msgs += int(r.trace[:, 2].sum())
        parts.append(f"{app} {r.supersteps} supersteps {r.seconds:.1f}s")
        print(f"[bench] oracle {app}: {r.supersteps} supersteps in {r.seconds:.1f}s on {threads} threads",
              file=sys.stderr, flush=True)
    info = host_info()
    return {"value": round(msgs / secs / 1e9, 5), "unit": "GTEPS", "cores": threads, "kind": "oracle",
            "sample": f"{name}: " + ", ".join(parts) + " (pull form, OpenMP default static schedule over "
                      f"{threads} threads; messages of the supersteps run / their time)",
            "nproc": info.get("nproc"), "cpu_model": info.get("cpu_model"), "ram_gib": info.get("ram_gib")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rmat-s26",
                    help="rmat-s26 (PageRank on the directed graph, CC/SSSP on its symmetrised form) or a single "
                         "graph for every application (rmat-s20-sym, rmat-s22-sym, grid4096-sc, rmat-s14-dir)")
    ap.add_argument("--secondary", default="rmat-s20-sym", help="second workload reported beside it ('none': skip)")
    ap.add_argument("--pr-updates", type=int, default=10)
    ap.add_argument("--mode", default="auto", help="exchange for CC/SSSP: auto, push or pull")
    ap.add_argument("--selector", default="learned", choices=["learned", "heuristic"],
                    help="what AUTO uses to pick the exchange: the trained network or the fixed rule")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--apps", default="pagerank,cc,sssp")
    ap.add_argument("--no-tune", action="store_true", help="run with the library's default launch parameters")
    ap.add_argument("--no-blocked", action="store_true",
                    help="build the graph without blocked in-edges (PageRank then pulls with the row-item kernels)")
    ap.add_argument("--binned", default="auto", choices=["auto", "on", "off"],
                    help="bin cold sources (auto: when the vertex-value array fills the 256 MB Infinity Cache)")
    ap.add_argument("--binned-hot", type=int, default=0, help="sources gathered edge by edge when binned (0: default)")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "_build", "tuning_cache.json"),
                    help="autotuner cache file")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched-vs-plain comparison (256-source SSSP on R-MAT s22 + 64 small PageRank graphs)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (to scale HBM byte counters), then exit")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU path is a design, "
              f"not implemented here", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import graphgen
    import paper_2010_08781_amd as ipg

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        n = args.calibrate_copy << 20
        x = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n, "copies": 3}), flush=True)
        return
    ipg.lib()
    apps = [a.strip() for a in args.apps.split(",") if a.strip()]
    T = args.pr_updates
    sel = None
    if args.selector == "learned" and args.mode == "auto":
        from paper_2010_08781_amd import selector_fit

        sel = selector_fit.load()
        if sel is None:
            sys.exit("bench.py: --selector learned but no trained selector parameters are installed")
    tune_cache = args.tune_cache

    main_w = bench_workload(args.workload, args, sel, ipg, np, torch, args.steps, args.warmup, apps, tune_cache)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.workload, main_w["host"], apps, T, np)
    for g in set(main_w.pop("graphs").values()):
        g.close()
    host_main = main_w.pop("host")
    n_pr, m_pr = host_main[apps[0]].n, host_main[apps[0]].m
    footprint = {a: {k: v for k, v in ipg.footprint(h.n, h.m, symmetric=bool(h.symmetric),
                                                    weighted=h.csr_w is not None, blocked=not args.no_blocked).items()
                     if k in ("total", "bytes_per_edge", "graph_workspace")}
                 for a, h in host_main.items()}
    del host_main
    torch.cuda.empty_cache()

    secondary = None
    if args.secondary and args.secondary != "none" and args.secondary != args.workload:
        sw = bench_workload(args.secondary, args, sel, ipg, np, torch, args.steps, min(args.warmup, 2), apps,
                            tune_cache)
        for g in set(sw.pop("graphs").values()):
            g.close()
        sw.pop("host")
        secondary = {k: sw[k] for k in ("name", "value", "ms_per_step", "apps", "learned_vs_plain", "roofline",
                                        "tuning")}
        secondary["value"] = round(secondary["value"], 4)
        secondary["ms_per_step"] = round(secondary["ms_per_step"], 4)
        torch.cuda.empty_cache()

    batched = None
    if not args.no_batched:
        batched = batched_vs_plain(ipg, graphgen, np, torch, tune_cache=None if args.no_tune else tune_cache)
        print(f"[bench] batched vs plain: {json.dumps(batched['end_to_end'])}", file=sys.stderr, flush=True)

    desc = (f"{args.workload}: PageRank T={T} pull FP64 on {main_w['apps'].get('pagerank', {}).get('graph', '-')}"
            f" + hash-min CC + SSSP from 0 on {main_w['apps'].get('cc', main_w['apps'].get('sssp', {})).get('graph', '-')},"
            f" exchange={args.mode}{' (trained selector)' if sel is not None else ''}, device-driven loop")
    line = {
        "metric": METRIC,
        "value": round(main_w["value"], 4),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_w["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+u32",
        "data": "synthetic",
        "config": {"workload": desc, "n": n_pr, "m": m_pr, "apps": main_w["apps"]},
        "tuning": main_w["tuning"],
        "footprint": footprint,
        "learned_vs_plain": main_w["learned_vs_plain"],
        "batched_vs_plain": batched,
        "secondary": secondary,
        "roofline": main_w["roofline"],
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
