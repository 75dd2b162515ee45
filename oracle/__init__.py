"""CPU oracle -- TEST INFRASTRUCTURE ONLY.

A plain sequential bulk-synchronous Pregel (oracle.c) that executes the
iPregel applications of Figs. 8-10 with naive vertex selection (Section 4.3.1)
and one-slot combining mailboxes (Section 4.3.3), and the same supersteps in
the pull form (Section 4.3.2) with the vertex loop under an OpenMP static
schedule (Section 4.2): `run_pull`, whose output does not depend on the
thread count and equals the push form's when the CSC lists are sorted.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package; the GPU library never does, and the two share no code.

Every function here is pinned by CPU tests against closed forms, invariants
and textbook routines (see tests/test_oracle_pins.py).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

APP_PAGERANK, APP_CC, APP_SSSP = 0, 1, 2
APPS = {"pagerank": APP_PAGERANK, "pr": APP_PAGERANK, "cc": APP_CC, "sssp": APP_SSSP}
OK, NOT_CONVERGED, EINVAL, EBADGRAPH, EOVERFLOW = 0, 1, -1, -2, -3
INF = 0xFFFFFFFF


def build(force: bool = False) -> str:
    """Compile oracle.c (gcc -O2, no FP contraction, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-Wall",
                               "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _L():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.orc_run.argtypes = [ctypes.c_int, ctypes.c_uint32, P, P, P, ctypes.c_uint32, ctypes.c_uint32,
                                P, P, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32)]
        lib.orc_run.restype = ctypes.c_int
        lib.orc_pagerank_deltas.argtypes = [ctypes.c_uint32, P, P, ctypes.c_uint32, ctypes.c_double, P, P]
        lib.orc_pagerank_deltas.restype = ctypes.c_int
        lib.orc_pagerank_run.argtypes = [ctypes.c_uint32, P, P, ctypes.c_uint32, ctypes.c_double, P, P,
                                         ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32)]
        lib.orc_pagerank_run.restype = ctypes.c_int
        lib.orc_run_pull.argtypes = [ctypes.c_int, ctypes.c_uint32, P, P, P, P, P, ctypes.c_uint32, ctypes.c_uint32,
                                     ctypes.c_double, ctypes.c_int, ctypes.c_int, P, P, ctypes.c_uint32,
                                     ctypes.POINTER(ctypes.c_uint32)]
        lib.orc_run_pull.restype = ctypes.c_int
        _lib = lib
    return _lib


@dataclass
class OracleResult:
    values: np.ndarray        # float64 (PageRank) or uint32 (CC, SSSP)
    trace: np.ndarray         # [supersteps, 3] uint64: active, senders, messages
    supersteps: int
    status: int
    seconds: float            # wall time of the superstep loop call


def run(app, n: int, csr_off: np.ndarray, csr_dst: np.ndarray, param: int, source: int = 0,
        csr_w=None, trace_cap: int = 1 << 16, damping: float = 0.85) -> OracleResult:
    """Run one application on a CSR graph held in host memory (push form,
    one thread).

    param: PageRank -> number of rank updates (the superstep at which
    vertices stop broadcasting, 10 in Fig. 8); CC/SSSP -> cap on the number
    of supersteps, 0 = unlimited.  damping: PageRank's d (ratio (1-d)/N).
    """
    app = APPS[app] if isinstance(app, str) else int(app)
    off = np.ascontiguousarray(csr_off, dtype=np.uint64)
    adj = np.ascontiguousarray(csr_dst, dtype=np.int32)
    if adj.size == 0:
        adj = np.zeros(1, dtype=np.int32)
    w = None if csr_w is None else np.ascontiguousarray(csr_w, dtype=np.uint32)
    if w is not None and w.size == 0:
        w = np.zeros(1, dtype=np.uint32)
    vals = np.zeros(max(n, 1), dtype=np.float64 if app == APP_PAGERANK else np.uint32)
    trace = np.zeros((trace_cap, 3), dtype=np.uint64)
    steps = ctypes.c_uint32(0)
    t0 = time.perf_counter()
    if app == APP_PAGERANK:
        st = _L().orc_pagerank_run(n, off.ctypes.data, adj.ctypes.data, param, float(damping), vals.ctypes.data,
                                   trace.ctypes.data, trace_cap, ctypes.byref(steps))
    else:
        st = _L().orc_run(app, n, off.ctypes.data, adj.ctypes.data, None if w is None else w.ctypes.data,
                          source, param, vals.ctypes.data, trace.ctypes.data, trace_cap, ctypes.byref(steps))
    dt = time.perf_counter() - t0
    k = min(int(steps.value), trace_cap)
    return OracleResult(values=vals[:n], trace=trace[:k].copy(), supersteps=int(steps.value), status=int(st),
                        seconds=dt)


def pagerank_deltas(n: int, csr_off, csr_dst, updates: int, damping: float = 0.85) -> np.ndarray:
    """L1 change of every update of Fig. 8's PageRank: out[s] = sum_v
    |r_s(v) - r_{s-1}(v)| for s = 1..updates (out[0] = 0)."""
    off = np.ascontiguousarray(csr_off, dtype=np.uint64)
    adj = np.ascontiguousarray(csr_dst, dtype=np.int32)
    if adj.size == 0:
        adj = np.zeros(1, dtype=np.int32)
    vals = np.zeros(max(n, 1), dtype=np.float64)
    d = np.zeros(updates + 1, dtype=np.float64)
    st = _L().orc_pagerank_deltas(n, off.ctypes.data, adj.ctypes.data, updates, float(damping), vals.ctypes.data,
                                  d.ctypes.data)
    assert st == OK, st
    return d


def pagerank_converge(g, tol: float, max_updates: int, damping: float = 0.85):
    """PageRank to convergence: stop after the first update s >= 1 whose L1
    change is below tol (or after max_updates).  Returns (result of the
    fixed run with T = that update, T, deltas)."""
    d = pagerank_deltas(g.n, g.csr_off, g.csr_dst, max_updates, damping)
    below = np.flatnonzero(d[1:] < tol)
    T = int(below[0]) + 1 if below.size else max_updates
    return run_graph("pagerank", g, T, damping=damping), T, d


def run_graph(app, g, param: int, source: int = 0, weighted: bool = True, trace_cap: int = 1 << 16,
              damping: float = 0.85):
    """Convenience wrapper for any object with n, csr_off, csr_dst, csr_w."""
    w = getattr(g, "csr_w", None) if weighted else None
    return run(app, g.n, g.csr_off, g.csr_dst, param, source=source, csr_w=w, trace_cap=trace_cap, damping=damping)


def run_pull(app, g, param: int, source: int = 0, weighted: bool = True, damping: float = 0.85,
             threads: int = 1, chunk: int = 0, trace_cap: int = 1 << 16) -> OracleResult:
    """The same run in the pull form, the vertex loop under an OpenMP static
    schedule over `threads` threads (0 = all the OpenMP runtime offers):
    chunk 0 = OpenMP's default static schedule (one contiguous block of
    vertices per thread, the paper's), else fixed chunks of that many
    vertices dealt round-robin.  The output is the same for any of them.
    `g` needs n, csr_off, csc_off, csc_src (and csr_w, csc_w when weighted)."""
    app = APPS[app] if isinstance(app, str) else int(app)
    n = int(g.n)
    roff = np.ascontiguousarray(g.csr_off, dtype=np.uint64)
    coff = np.ascontiguousarray(g.csc_off, dtype=np.uint64)
    src = np.ascontiguousarray(g.csc_src, dtype=np.int32)
    if src.size == 0:
        src = np.zeros(1, dtype=np.int32)
    rw = getattr(g, "csr_w", None) if weighted else None
    cw = getattr(g, "csc_w", None) if weighted else None
    if (rw is None) != (cw is None):
        raise ValueError("weights must be given for both orientations")
    rw = None if rw is None else np.ascontiguousarray(rw, dtype=np.uint32)
    cw = None if cw is None else np.ascontiguousarray(cw, dtype=np.uint32)
    if threads <= 0:
        threads = max_threads()
    vals = np.zeros(max(n, 1), dtype=np.float64 if app == APP_PAGERANK else np.uint32)
    trace = np.zeros((trace_cap, 3), dtype=np.uint64)
    steps = ctypes.c_uint32(0)
    t0 = time.perf_counter()
    st = _L().orc_run_pull(app, n, roff.ctypes.data, None if rw is None or rw.size == 0 else rw.ctypes.data,
                           coff.ctypes.data, src.ctypes.data, None if cw is None or cw.size == 0 else cw.ctypes.data,
                           source, param, float(damping), int(threads), int(chunk), vals.ctypes.data,
                           trace.ctypes.data,
                           trace_cap, ctypes.byref(steps))
    dt = time.perf_counter() - t0
    k = min(int(steps.value), trace_cap)
    return OracleResult(values=vals[:n], trace=trace[:k].copy(), supersteps=int(steps.value), status=int(st),
                        seconds=dt)


def max_threads() -> int:
    """Threads the OpenMP runtime of the oracle offers (OMP_NUM_THREADS or the cores)."""
    lib = _L()
    if not hasattr(lib, "_mt"):
        lib.orc_max_threads.argtypes = []
        lib.orc_max_threads.restype = ctypes.c_int
        lib._mt = True
    return int(lib.orc_max_threads())
