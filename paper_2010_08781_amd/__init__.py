"""Python binding of the gfx950 superstep engine (libipregel.so).

Argument marshalling only: every superstep runs in the library's HIP kernels.
PyTorch provides device memory (graph arrays, workspaces, outputs) and the
stream; the library never allocates device memory.

    import paper_2010_08781_amd as ipg
    g = ipg.Graph.from_csr_csc(n, csr_off, csr_dst, csc_off, csc_src)   # torch cuda tensors
    ranks, stats = g.run("pagerank", 10)
    labels, stats = g.run("cc")
    dist, stats = g.run("sssp", source=0)

The applications are those of the iPregel paper (Section 6): PageRank
(Fig. 8, sum combiner), hash-min connected components (Fig. 9) and SSSP
(Fig. 10), both with the min combiner.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libipregel.so")

OK, NOT_CONVERGED = 0, 1
EINVAL, EBADGRAPH, EUNSUPPORTED, EWORKSPACE, EDEVICE, EOVERFLOW = -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "IPG_OK", 1: "IPG_NOT_CONVERGED", -1: "IPG_EINVAL", -2: "IPG_EBADGRAPH", -3: "IPG_EUNSUPPORTED",
                -4: "IPG_EWORKSPACE", -5: "IPG_EDEVICE", -6: "IPG_EOVERFLOW"}
APP_PAGERANK, APP_CC, APP_SSSP = 0, 1, 2
APPS = {"pagerank": APP_PAGERANK, "pr": APP_PAGERANK, "cc": APP_CC, "sssp": APP_SSSP}
COMBINE_SUM, COMBINE_MIN = 0, 1
DEFAULT_COMBINER = {APP_PAGERANK: COMBINE_SUM, APP_CC: COMBINE_MIN, APP_SSSP: COMBINE_MIN}
MODES = {"auto": 0, "push": 1, "pull": 2}
GRAPH_SYMMETRIC, GRAPH_VALIDATE, GRAPH_RENAME, GRAPH_BLOCKED, GRAPH_BINNED = 1, 2, 4, 8, 16
RUN_PERSISTENT, RUN_GRAPH, RUN_ENQUEUE = 1, 2, 4
INF = 0xFFFFFFFF
BATCH_MAX_SOURCES = 256


class IpgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class _Desc(ctypes.Structure):
    _fields_ = [("num_vertices", ctypes.c_uint32), ("num_edges", ctypes.c_uint64),
                ("csr_off", ctypes.c_void_p), ("csr_dst", ctypes.c_void_p),
                ("csc_off", ctypes.c_void_p), ("csc_src", ctypes.c_void_p),
                ("csr_w", ctypes.c_void_p), ("csc_w", ctypes.c_void_p), ("flags", ctypes.c_uint32),
                ("binned_hot", ctypes.c_uint32)]


class _Tuning(ctypes.Structure):
    _fields_ = [("pr_hot", ctypes.c_uint32), ("pull_grid", ctypes.c_uint32), ("push_div", ctypes.c_uint32),
                ("list_div", ctypes.c_uint32), ("gate_div", ctypes.c_uint32), ("blocked", ctypes.c_uint32),
                ("late_div", ctypes.c_uint32)]


TUNING_FIELDS = ("pr_hot", "pull_grid", "push_div", "list_div", "gate_div", "blocked", "late_div")
HOT_OFF = 0xFFFFFFFF


def _tuning(t):
    if t is None:
        return None
    unknown = set(t) - set(TUNING_FIELDS)
    if unknown:
        raise ValueError(f"unknown tuning fields {sorted(unknown)}")
    return _Tuning(*(int(t.get(k, 0)) for k in TUNING_FIELDS))


class _Opts(ctypes.Structure):
    _fields_ = [("source", ctypes.c_uint32), ("damping", ctypes.c_double), ("mode", ctypes.c_int),
                ("flags", ctypes.c_uint32),
                ("selector", ctypes.c_void_p), ("part_offsets", ctypes.c_void_p), ("num_parts", ctypes.c_uint32),
                ("tolerance", ctypes.c_double), ("tuning", ctypes.c_void_p)]


class _Stats(ctypes.Structure):
    _fields_ = [("supersteps", ctypes.c_uint32), ("halted", ctypes.c_uint32),
                ("edges_traversed", ctypes.c_uint64), ("edges_examined", ctypes.c_uint64),
                ("seconds", ctypes.c_double), ("trace_cap", ctypes.c_uint32),
                ("active", ctypes.c_void_p), ("senders", ctypes.c_void_p), ("messages", ctypes.c_void_p),
                ("examined", ctypes.c_void_p), ("mode", ctypes.c_void_p), ("usec", ctypes.c_void_p),
                ("frontier_deg", ctypes.c_void_p), ("residual", ctypes.c_void_p)]


_lib = None


def lib():
    """Load libipregel.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        # PyTorch ships its own HIP runtime under the same soname; importing
        # it first makes the library bind to that runtime instead of loading
        # a second one into the process (two runtimes do not share the GPU).
        import torch  # noqa: F401

        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it first (python __graft_entry__.py or "
                              f"python paper_2010_08781_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        P, u32, u64, i32, sz = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_size_t
        L.ipg_graph_workspace_bytes.argtypes = [u32, u64, u32]
        L.ipg_graph_workspace_bytes.restype = sz
        L.ipg_run_workspace_bytes.argtypes = [u32, u64, i32]
        L.ipg_run_workspace_bytes.restype = sz
        L.ipg_graph_create.argtypes = [ctypes.POINTER(_Desc), P, sz, P, ctypes.POINTER(P)]
        L.ipg_graph_create.restype = i32
        L.ipg_run.argtypes = [P, i32, i32, u32, ctypes.POINTER(_Opts), P, sz, P, ctypes.POINTER(_Stats)]
        L.ipg_run.restype = i32
        L.ipg_read_values.argtypes = [P, P, sz, i32, P]
        L.ipg_read_values.restype = i32
        L.ipg_graph_destroy.argtypes = [P]
        L.ipg_graph_destroy.restype = None
        L.ipg_last_error.argtypes = []
        L.ipg_last_error.restype = ctypes.c_char_p
        L.ipg_multi_sssp_workspace_bytes.argtypes = [u32, u64]
        L.ipg_multi_sssp_workspace_bytes.restype = sz
        L.ipg_run_multi_sssp.argtypes = [P, P, u32, u32, ctypes.POINTER(_Opts), P, sz, P, sz, P, ctypes.POINTER(_Stats)]
        L.ipg_run_multi_sssp.restype = i32
        L.ipg_multi_sssp_result.argtypes = [P, P, sz, P, ctypes.POINTER(_Stats)]
        L.ipg_multi_sssp_result.restype = i32
        L.ipg_selector_workspace_bytes.argtypes = [u32]
        L.ipg_selector_workspace_bytes.restype = sz
        L.ipg_selector_forward.argtypes = [P, P, u32, P, P]
        L.ipg_selector_forward.restype = i32
        L.ipg_selector_grad.argtypes = [P, P, P, u32, P, P, sz, P]
        L.ipg_selector_grad.restype = i32
        L.ipg_selector_train.argtypes = [P, P, P, u32, u32, ctypes.c_double, P, sz, P]
        L.ipg_selector_train.restype = i32
        L.ipg_selector_train_noalloc.argtypes = [P, P, P, u32, u32, ctypes.c_double, P]
        L.ipg_selector_train_noalloc.restype = i32
        _lib = L
    return _lib


def last_error() -> str:
    return lib().ipg_last_error().decode()


def _check(st: int, what: str, allow_not_converged: bool = False) -> int:
    if st == OK or (allow_not_converged and st == NOT_CONVERGED):
        return st
    raise IpgError(st, f"{what}: {last_error()}")


def _stream_handle(stream=None) -> int:
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


@dataclass
class RunStats:
    status: int
    supersteps: int
    halted: bool
    edges_traversed: int
    edges_examined: int
    seconds: float
    active: np.ndarray = field(repr=False)
    senders: np.ndarray = field(repr=False)
    messages: np.ndarray = field(repr=False)
    examined: np.ndarray = field(repr=False)
    mode: np.ndarray = field(repr=False)
    usec: Optional[np.ndarray] = field(repr=False, default=None)
    frontier_deg: Optional[np.ndarray] = field(repr=False, default=None)
    residual: Optional[np.ndarray] = field(repr=False, default=None)

    @property
    def trace(self) -> np.ndarray:
        """[supersteps, 3] uint64: active, senders, messages (the oracle's trace layout)."""
        return np.stack([self.active, self.senders, self.messages], axis=1)

    @property
    def gteps(self) -> float:
        return self.edges_traversed / self.seconds / 1e9 if self.seconds > 0 else float("nan")


class _Trace:
    """Host arrays for ipg_run_stats and their conversion to RunStats."""

    def __init__(self, cap: int, timing: bool):
        self.cap = cap
        self.last = 0  # supersteps the previous run filled (for reuse)
        self.a = {k: np.zeros(cap, dtype=np.uint64) for k in ("active", "senders", "messages", "examined", "frontier_deg")}
        self.a["mode"] = np.zeros(cap, dtype=np.uint8)
        self.usec = np.zeros(cap, dtype=np.float32) if timing else None
        self.residual = np.zeros(cap, dtype=np.float64)
        a = self.a
        self.st = _Stats(0, 0, 0, 0, 0.0, cap, a["active"].ctypes.data, a["senders"].ctypes.data,
                         a["messages"].ctypes.data, a["examined"].ctypes.data, a["mode"].ctypes.data,
                         self.usec.ctypes.data if self.usec is not None else None, a["frontier_deg"].ctypes.data,
                         self.residual.ctypes.data)

    def reset(self):
        """Prepare the buffers for another run: clear the entries a run may
        leave unwritten (per-superstep times, residuals) up to the previous
        run's length."""
        k = self.last
        if k:
            if self.usec is not None:
                self.usec[:k] = 0
            self.residual[:k] = 0
        st = self.st
        st.supersteps = st.halted = st.edges_traversed = st.edges_examined = 0
        st.seconds = 0.0
        return self

    def stats(self, rc: int) -> "RunStats":
        st, a = self.st, self.a
        if rc not in (OK, NOT_CONVERGED):
            return RunStats(rc, 0, False, 0, 0, 0.0, *(np.zeros(0),) * 5)
        k = min(int(st.supersteps), self.cap)
        self.last = max(self.last, k)
        # copies: the buffers are reused by the next run on the graph
        return RunStats(rc, int(st.supersteps), bool(st.halted), int(st.edges_traversed), int(st.edges_examined),
                        float(st.seconds), a["active"][:k].copy(), a["senders"][:k].copy(), a["messages"][:k].copy(),
                        a["examined"][:k].copy(), a["mode"][:k].copy(),
                        self.usec[:k].copy() if self.usec is not None else None, a["frontier_deg"][:k].copy(),
                        self.residual[:k].copy())


class Graph:
    """A graph resident on the current HIP device (CSR + CSC held as torch tensors)."""

    def __init__(self, n, csr_off, csr_dst, csc_off=None, csc_src=None, csr_w=None, csc_w=None,
                 symmetric=False, validate=True, stream=None, rename=True, blocked=False, binned=False,
                 binned_hot: int = 0):
        import torch

        self.n = int(n)
        self.m = int(csr_dst.numel())
        self.symmetric = bool(symmetric)
        if symmetric:
            csc_off = csr_off if csc_off is None else csc_off
            csc_src = csr_dst if csc_src is None else csc_src
            csc_w = csr_w if csc_w is None else csc_w
        for name, t, dt in (("csr_off", csr_off, torch.int64), ("csr_dst", csr_dst, torch.int32),
                            ("csc_off", csc_off, torch.int64), ("csc_src", csc_src, torch.int32)):
            if t is None or not t.is_cuda or t.dtype != dt or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous {dt} CUDA tensor")
        for name, t in (("csr_w", csr_w), ("csc_w", csc_w)):
            if t is not None and (not t.is_cuda or t.dtype not in (torch.int32, torch.uint32) or not t.is_contiguous()):
                raise ValueError(f"{name} must be a contiguous 32-bit integer CUDA tensor")
        if csr_off.numel() != self.n + 1 or csc_off.numel() != self.n + 1:
            raise ValueError("offset arrays must have n+1 entries")
        if csc_src.numel() != self.m:
            raise ValueError("CSR and CSC must hold the same number of edges")
        # keep caller tensors alive for the lifetime of the handle
        self._keep = (csr_off, csr_dst, csc_off, csc_src, csr_w, csc_w)
        self.weighted = csr_w is not None
        self.renamed = bool(rename)
        self.blocked = bool(blocked or binned)
        self.binned = bool(binned)
        flags = (GRAPH_SYMMETRIC if symmetric else 0) | (GRAPH_VALIDATE if validate else 0) | \
            (GRAPH_RENAME if rename else 0) | (GRAPH_BLOCKED if self.blocked else 0) | (GRAPH_BINNED if binned else 0)
        d = _Desc(self.n, self.m, csr_off.data_ptr(), csr_dst.data_ptr() if self.m else None,
                  csc_off.data_ptr(), csc_src.data_ptr() if self.m else None,
                  csr_w.data_ptr() if csr_w is not None else None,
                  csc_w.data_ptr() if csc_w is not None else None, flags, int(binned_hot))
        nbytes = lib().ipg_graph_workspace_bytes(self.n, self.m, flags)
        self._gws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=csr_off.device)
        h = ctypes.c_void_p()
        _check(lib().ipg_graph_create(ctypes.byref(d), self._gws.data_ptr(), nbytes, _stream_handle(stream),
                                      ctypes.byref(h)), "ipg_graph_create")
        self._h = h
        self.device = csr_off.device
        self._run_ws = {}
        self._traces = {}

    @classmethod
    def from_csr_csc(cls, *args, **kw) -> "Graph":
        return cls(*args, **kw)

    @classmethod
    def from_host(cls, hg, device="cuda", validate=True, weighted=True, rename=True, blocked=False, binned=False,
                  binned_hot: int = 0) -> "Graph":
        """Upload any object with n, csr_off, csr_dst, csc_off, csc_src (numpy) and optional csr_w/csc_w."""
        import torch

        def up(a, dt):
            return torch.from_numpy(np.ascontiguousarray(a).view(dt)).to(device)

        csr_off = up(hg.csr_off.astype(np.uint64), np.int64)
        csr_dst = up(hg.csr_dst.astype(np.int32), np.int32)
        sym = bool(getattr(hg, "symmetric", False))
        if sym:
            csc_off, csc_src = csr_off, csr_dst
        else:
            csc_off = up(hg.csc_off.astype(np.uint64), np.int64)
            csc_src = up(hg.csc_src.astype(np.int32), np.int32)
        csr_w = csc_w = None
        if weighted and getattr(hg, "csr_w", None) is not None:
            csr_w = up(hg.csr_w.astype(np.uint32), np.int32)
            csc_w = csr_w if sym else up(hg.csc_w.astype(np.uint32), np.int32)
        return cls(hg.n, csr_off, csr_dst, csc_off, csc_src, csr_w, csc_w, symmetric=sym, validate=validate,
                   rename=rename, blocked=blocked, binned=binned, binned_hot=binned_hot)

    def _trace(self, cap: int, timing: bool) -> "_Trace":
        """The host trace buffers of this graph's runs (kept and reused: a
        fresh set per run cost measurable host time)."""
        key = (int(cap), bool(timing))
        if key not in self._traces:
            self._traces[key] = _Trace(cap, timing)
        return self._traces[key].reset()

    def workspace(self, app: int):
        import torch

        if app not in self._run_ws:
            nbytes = lib().ipg_run_workspace_bytes(self.n, self.m, app)
            self._run_ws[app] = (torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device), nbytes)
        return self._run_ws[app]

    def run(self, app, max_supersteps: Optional[int] = None, source: int = 0, mode: str = "auto",
            timing: bool = True, trace_cap: int = 1 << 16, persistent: bool = False, stream=None,
            combiner: Optional[int] = None, check: bool = True, selector=None, parts=None, graph: bool = False,
            tol: float = 0.0, tuning: Optional[dict] = None, enqueue: bool = False, damping: float = 0.0):
        """Run an application; returns (values tensor on the device, RunStats).

        max_supersteps: PageRank -> number of rank updates (default 10, Fig. 8);
        CC/SSSP -> cap on supersteps (default 0 = run to vote-to-halt).
        parts: PageRank over a disjoint union -- int32 CUDA tensor of part
        vertex offsets (P+1 entries); graph: replay PageRank as one hipGraph;
        tol: PageRank to convergence (stop after the first update whose L1
        change is below tol; max_supersteps caps the updates); tuning: launch
        parameters (see TUNING_FIELDS and the autotune module); enqueue:
        PageRank work only enqueued on the stream (capturable; returns
        (None, None), read the ranks with read_values afterwards); damping:
        PageRank's d (0 = 0.85, Fig. 8)."""
        import torch

        a = APPS[app] if isinstance(app, str) else int(app)
        if max_supersteps is None:
            max_supersteps = 10 if a == APP_PAGERANK else 0
        comb = DEFAULT_COMBINER.get(a, 0) if combiner is None else combiner
        ws, nbytes = self.workspace(a) if a in DEFAULT_COMBINER else (None, 0)
        if selector is not None:
            _check_selector(selector)
        if parts is not None:
            import torch

            if not parts.is_cuda or parts.dtype != torch.int32 or not parts.is_contiguous() or parts.numel() < 2:
                raise ValueError("parts must be a contiguous int32 CUDA tensor of P+1 offsets")
        flags = (RUN_PERSISTENT if persistent else 0) | (RUN_GRAPH if graph else 0) | (RUN_ENQUEUE if enqueue else 0)
        tun = _tuning(tuning)
        opts = _Opts(int(source), float(damping), MODES[mode], flags,
                     selector.data_ptr() if selector is not None else None,
                     parts.data_ptr() if parts is not None else None, parts.numel() - 1 if parts is not None else 0,
                     float(tol), ctypes.addressof(tun) if tun is not None else None)
        tr = self._trace(trace_cap, timing)
        sh = _stream_handle(stream)
        rc = lib().ipg_run(self._h, a, comb, int(max_supersteps), ctypes.byref(opts),
                           ws.data_ptr() if ws is not None else None, nbytes, sh,
                           None if enqueue else ctypes.byref(tr.st))
        if enqueue:
            _check(rc, "ipg_run")
            return None, None
        if check:
            _check(rc, "ipg_run", allow_not_converged=True)
        elif rc not in (OK, NOT_CONVERGED):
            return None, tr.stats(rc)
        vals = self._values(a, sh, stream)
        return vals, tr.stats(rc)

    def run_multi_sssp(self, sources, max_supersteps: int = 0, mode: str = "auto", timing: bool = True,
                       trace_cap: int = 1 << 16, stream=None, out=None, check: bool = True,
                       tuning: Optional[dict] = None, persistent: bool = False, enqueue: bool = False):
        """Batched unit-weight SSSP from up to 256 sources in one superstep loop.

        Returns (dist [Q, N] int32 tensor holding uint32 distances, RunStats whose
        trace is the sum of the single-source traces).  persistent: the loop
        runs on the device; enqueue: the device-driven run is only enqueued
        (capturable; stats None -- see multi_sssp_result)."""
        import torch

        src = torch.as_tensor(np.asarray(sources, dtype=np.int64).astype(np.int32), device=self.device) \
            if not torch.is_tensor(sources) else sources.to(device=self.device, dtype=torch.int32).contiguous()
        q = int(src.numel())
        if out is None:
            out = torch.empty((q, self.n), dtype=torch.int32, device=self.device)
        key = "multi_sssp"
        if key not in self._run_ws:
            nb = lib().ipg_multi_sssp_workspace_bytes(self.n, self.m)
            self._run_ws[key] = (torch.empty(max(nb, 256), dtype=torch.uint8, device=self.device), nb)
        ws, nbytes = self._run_ws[key]
        tun = _tuning(tuning)
        flags = (RUN_PERSISTENT if persistent else 0) | (RUN_ENQUEUE if enqueue else 0)
        opts = _Opts(0, 0.0, MODES[mode], flags, None, None, 0, 0.0,
                     ctypes.addressof(tun) if tun is not None else None)
        tr = self._trace(trace_cap, timing)
        self._ms_src = src  # the device ids must outlive an enqueued run
        rc = lib().ipg_run_multi_sssp(self._h, src.data_ptr(), q, int(max_supersteps), ctypes.byref(opts),
                                      out.data_ptr(), out.numel() * 4, ws.data_ptr(), nbytes, _stream_handle(stream),
                                      None if enqueue else ctypes.byref(tr.st))
        if enqueue:
            _check(rc, "ipg_run_multi_sssp")
            return out, None
        if check:
            _check(rc, "ipg_run_multi_sssp", allow_not_converged=True)
        return out, tr.stats(rc)

    def multi_sssp_result(self, trace_cap: int = 1024, stream=None, check: bool = True):
        """RunStats of the last device-driven batched run (after an enqueued run executed)."""
        ws, nbytes = self._run_ws["multi_sssp"]
        tr = self._trace(trace_cap, True)
        rc = lib().ipg_multi_sssp_result(self._h, ws.data_ptr(), nbytes, _stream_handle(stream), ctypes.byref(tr.st))
        if check:
            _check(rc, "ipg_multi_sssp_result", allow_not_converged=True)
        return tr.stats(rc)

    def read_values(self, app: int, stream=None):
        return self._values(app, _stream_handle(stream), stream)

    def _values(self, app: int, sh: int, stream):
        import torch

        dt = torch.float64 if app == APP_PAGERANK else torch.int32
        out = torch.empty(self.n, dtype=dt, device=self.device)
        _check(lib().ipg_read_values(self._h, out.data_ptr(), out.numel() * out.element_size(), 1, sh),
               "ipg_read_values")
        if stream is not None:  # the copy is enqueued on `stream`: order torch's current stream after it
            torch.cuda.current_stream().wait_stream(stream)
        return out

    def close(self):
        if getattr(self, "_h", None):
            lib().ipg_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------ selector ----

SELECTOR_PARAMS, SELECTOR_INPUTS, SELECTOR_OUTPUTS = 403, 4, 3


def _check_selector(p):
    import torch

    if not p.is_cuda or p.dtype != torch.float64 or p.numel() != SELECTOR_PARAMS or not p.is_contiguous():
        raise ValueError(f"selector parameters must be a contiguous float64 CUDA tensor of {SELECTOR_PARAMS}")


def _check_batch(x, t=None):
    import torch

    if not x.is_cuda or x.dtype != torch.float64 or x.dim() != 2 or x.shape[1] != SELECTOR_INPUTS:
        raise ValueError("selector inputs must be a float64 CUDA tensor [n, 4]")
    if t is not None and (not t.is_cuda or t.dtype != torch.float64 or tuple(t.shape) != (x.shape[0], SELECTOR_OUTPUTS)):
        raise ValueError("selector targets must be a float64 CUDA tensor [n, 2]")


def selector_forward(params, x, stream=None):
    """Predicted log2-times [n, 2] (push, pull) for inputs x [n, 4]."""
    import torch

    _check_selector(params)
    _check_batch(x)
    x = x.contiguous()
    y = torch.empty((x.shape[0], SELECTOR_OUTPUTS), dtype=torch.float64, device=x.device)
    _check(lib().ipg_selector_forward(params.data_ptr(), x.data_ptr(), x.shape[0], y.data_ptr(),
                                      _stream_handle(stream)), "ipg_selector_forward")
    return y


def _selector_ws(n, device):
    import torch

    nbytes = lib().ipg_selector_workspace_bytes(n)
    return torch.empty(nbytes, dtype=torch.uint8, device=device), nbytes


def selector_grad(params, x, t, stream=None):
    """Gradient of (1/2n) sum (y - t)^2 with respect to the parameters."""
    import torch

    _check_selector(params)
    _check_batch(x, t)
    x, t = x.contiguous(), t.contiguous()
    g = torch.empty(SELECTOR_PARAMS, dtype=torch.float64, device=x.device)
    ws, nbytes = _selector_ws(x.shape[0], x.device)
    _check(lib().ipg_selector_grad(params.data_ptr(), x.data_ptr(), t.data_ptr(), x.shape[0], g.data_ptr(),
                                   ws.data_ptr(), nbytes, _stream_handle(stream)), "ipg_selector_grad")
    return g


def selector_train(params, x, t, epochs: int, lr: float, stream=None):
    """In-place full-batch gradient descent on the device."""
    _check_selector(params)
    _check_batch(x, t)
    x, t = x.contiguous(), t.contiguous()
    ws, nbytes = _selector_ws(x.shape[0], x.device)
    _check(lib().ipg_selector_train(params.data_ptr(), x.data_ptr(), t.data_ptr(), x.shape[0], int(epochs), float(lr),
                                    ws.data_ptr(), nbytes, _stream_handle(stream)), "ipg_selector_train")
    return params


SELECTOR_NOALLOC_MAX_SAMPLES = 16384


def selector_train_noalloc(params, x, t, epochs: int, lr: float, stream=None):
    """ipg_selector_train_noalloc: the same training with the library's
    static scratch instead of a workspace (no device allocation)."""
    _check_selector(params)
    _check_batch(x, t)
    if not (x.is_contiguous() and t.is_contiguous()):
        raise ValueError("selector inputs and targets must be contiguous (no copies are made)")
    _check(lib().ipg_selector_train_noalloc(params.data_ptr(), x.data_ptr(), t.data_ptr(), x.shape[0], int(epochs),
                                            float(lr), _stream_handle(stream)), "ipg_selector_train_noalloc")
    return params


def selector_features(frontier, frontier_deg, superstep, num_edges) -> np.ndarray:
    """The network's inputs for superstep states (same definition as the library's)."""
    f = np.asarray(frontier, dtype=np.float64)
    d = np.asarray(frontier_deg, dtype=np.float64)
    s = np.minimum(np.asarray(superstep, dtype=np.float64), 128.0)
    e = np.broadcast_to(np.asarray(num_edges, dtype=np.float64), f.shape)
    return np.stack([np.log2(1 + f) / 32, np.log2(1 + d) / 32, s / 64, np.log2(1 + e) / 32], axis=-1)


def values_to_numpy(t) -> np.ndarray:
    """Device values -> numpy (uint32 view for CC/SSSP, float64 for PageRank)."""
    import torch

    a = t.cpu().numpy()
    return a.view(np.uint32) if t.dtype == torch.int32 else a


# ----------------------------------------------------------- footprint ----

def footprint(n: int, m: int, symmetric: bool = False, weighted: bool = False, rename: bool = True,
              blocked: bool = False, binned: bool = False) -> dict:
    """Device memory of a graph and of each application's run, in bytes
    (the library's own size queries plus the caller-owned graph arrays):
    the device-side counterpart of the paper's memory-usage comparison
    (Table 3).  A symmetric graph stores one adjacency (CSC aliases CSR)."""
    L = lib()
    flags = (GRAPH_SYMMETRIC if symmetric else 0) | (GRAPH_RENAME if rename else 0) | \
        (GRAPH_BLOCKED if blocked or binned else 0) | (GRAPH_BINNED if binned else 0)
    adj = 8 * (n + 1) + 4 * m
    arrays = {"csr": adj, "csc": 0 if symmetric else adj,
              "weights": (4 * m if symmetric else 8 * m) if weighted else 0}
    graph_ws = int(L.ipg_graph_workspace_bytes(n, m, flags))
    base = sum(arrays.values()) + graph_ws
    runs = {name: int(L.ipg_run_workspace_bytes(n, m, app)) for name, app in
            (("pagerank", APP_PAGERANK), ("cc", APP_CC), ("sssp", APP_SSSP))}
    runs["multi_sssp"] = int(L.ipg_multi_sssp_workspace_bytes(n, m))
    out = {"n": n, "m": m, "symmetric": symmetric, "weighted": weighted, "rename": rename, "blocked": blocked,
           "binned": binned,
           "graph_arrays": arrays,
           "graph_workspace": graph_ws, "run_workspace": runs,
           "total": {k: base + v for k, v in runs.items()}}
    out["bytes_per_edge"] = {k: round(v / max(m, 1), 3) for k, v in out["total"].items()}
    out["bytes_per_vertex_run"] = {k: round(v / max(n, 1), 3) for k, v in runs.items()}
    return out
