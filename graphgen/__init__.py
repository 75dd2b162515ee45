"""Seeded synthetic graph inputs shared by the CPU oracle and the GPU library.

This package generates graphs and assembles them into CSR (out-adjacency) and
CSC (in-adjacency) arrays.  It contains none of the vertex-centric method's
arithmetic, so both sides of every parity test can consume its output without
sharing any code with each other.

Workloads (stand-ins for the paper's SNAP graphs, Table 1, which are not
available here):

* R-MAT (Chakrabarti et al., SDM 2004), (a,b,c,d) = (0.57, 0.19, 0.19, 0.05),
  edge factor 16, self-loops and duplicates removed, optionally symmetrised.
  The skewed degree distribution mimics the social graphs of Table 1.
* A square 4-neighbour grid with 1 % random long-range shortcuts and integer
  weights in [1, 255], a high-diameter weighted SSSP input.
* Families of small R-MAT graphs of uneven size.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")

RMAT_ABC = (0.57, 0.19, 0.19)


def build(force: bool = False) -> str:
    """Compile graphgen.c into libgraphgen.so (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", "-o", tmp, _SRC]
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _L():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        u64, u32, i32, dbl = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_double
        lib.gg_rmat_edges.argtypes = [i32, u64, dbl, dbl, dbl, u64, P, P]
        lib.gg_rmat_edges.restype = None
        lib.gg_rmat_edges_bounded.argtypes = [i32, u32, u64, dbl, dbl, dbl, u64, P, P]
        lib.gg_rmat_edges_bounded.restype = u64
        lib.gg_build_csr.argtypes = [u32, u64, P, P, i32, P, P]
        lib.gg_build_csr.restype = u64
        lib.gg_transpose.argtypes = [u32, P, P, P, P]
        lib.gg_transpose.restype = None
        lib.gg_symmetrise.argtypes = [u32, P, P, P, P, P, P]
        lib.gg_symmetrise.restype = u64
        lib.gg_edge_weights.argtypes = [u32, P, P, u64, u32, u32, P]
        lib.gg_edge_weights.restype = None
        lib.gg_grid_edges.argtypes = [u32, u32, P, P]
        lib.gg_grid_edges.restype = u64
        lib.gg_grid_shortcuts.argtypes = [u32, u32, u64, u64, P, P]
        lib.gg_grid_shortcuts.restype = None
        lib.gg_pick_sources.argtypes = [u32, P, u64, u64, P]
        lib.gg_pick_sources.restype = None
        lib.gg_splitmix_draw.argtypes = [u64, u64, u64]
        lib.gg_splitmix_draw.restype = u64
        lib.gg_max_threads.argtypes = []
        lib.gg_max_threads.restype = i32
        _lib = lib
    return _lib


def _p(a: np.ndarray) -> ctypes.c_void_p:
    assert a.flags["C_CONTIGUOUS"]
    return ctypes.c_void_p(a.ctypes.data)


@dataclass
class HostGraph:
    """A graph in host memory: CSR out-adjacency plus CSC in-adjacency.

    ids are int32 in [0, n); offsets are uint64 with off[0] == 0 and
    off[n] == m.  Lists are sorted ascending.  For a symmetric graph the CSC
    arrays are the CSR arrays (same objects).  Weights, when present, are
    uint32 aligned with the adjacency arrays.
    """

    n: int
    csr_off: np.ndarray
    csr_dst: np.ndarray
    csc_off: np.ndarray
    csc_src: np.ndarray
    symmetric: bool = False
    csr_w: Optional[np.ndarray] = None
    csc_w: Optional[np.ndarray] = None
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.csr_off[-1])

    @property
    def outdeg(self) -> np.ndarray:
        return np.diff(self.csr_off).astype(np.uint32)

    @property
    def indeg(self) -> np.ndarray:
        return np.diff(self.csc_off).astype(np.uint32)

    def summary(self) -> dict:
        od, idg = np.diff(self.csr_off), np.diff(self.csc_off)
        return {
            "name": self.name,
            "n": self.n,
            "m": self.m,
            "symmetric": self.symmetric,
            "weighted": self.csr_w is not None,
            "dangling": int((od == 0).sum()),
            "no_in_edges": int((idg == 0).sum()),
            "max_outdeg": int(od.max()) if self.n else 0,
            "max_indeg": int(idg.max()) if self.n else 0,
        }


def _csr_from_edges(n: int, src: np.ndarray, dst: np.ndarray, symmetric: bool, keep_loops: bool,
                    keep_dups: bool):
    src = np.ascontiguousarray(src, dtype=np.uint32)
    dst = np.ascontiguousarray(dst, dtype=np.uint32)
    flags = (1 if symmetric else 0) | (2 if keep_loops else 0) | (4 if keep_dups else 0)
    off = np.zeros(n + 1, dtype=np.uint64)
    cap = _L().gg_build_csr(n, src.size, _p(src), _p(dst), flags, _p(off), None)
    adj = np.empty(max(int(cap), 1), dtype=np.int32)
    m = _L().gg_build_csr(n, src.size, _p(src), _p(dst), flags, _p(off), _p(adj))
    return off, adj[: int(m)].copy() if m < adj.size else adj[: int(m)]


def _transpose(n: int, off: np.ndarray, adj: np.ndarray):
    toff = np.zeros(n + 1, dtype=np.uint64)
    tadj = np.empty(max(adj.size, 1), dtype=np.int32)
    _L().gg_transpose(n, _p(off), _p(adj if adj.size else np.zeros(1, np.int32)), _p(toff), _p(tadj))
    return toff, tadj[: adj.size]


def _weights(n, off, adj, seed, lo, hi):
    w = np.empty(max(adj.size, 1), dtype=np.uint32)
    _L().gg_edge_weights(n, _p(off), _p(adj if adj.size else np.zeros(1, np.int32)), seed, lo, hi, _p(w))
    return w[: adj.size]


def from_edges(n: int, src, dst, symmetric: bool = False, keep_self_loops: bool = False,
               keep_duplicates: bool = False, weight_seed: Optional[int] = None,
               wmin: int = 1, wmax: int = 255, name: str = "edges") -> HostGraph:
    """Assemble a HostGraph from an edge list (edges with an end >= n are dropped).

    With symmetric=True every edge is also added reversed and the CSC aliases
    the CSR.  Weights, when weight_seed is given, depend only on the unordered
    endpoint pair, so an undirected edge carries the same weight both ways.
    """
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    assert src.shape == dst.shape
    assert (src >= 0).all() and (dst >= 0).all()
    off, adj = _csr_from_edges(n, src.astype(np.uint32), dst.astype(np.uint32), symmetric,
                               keep_self_loops, keep_duplicates)
    if symmetric:
        toff, tadj = off, adj
    else:
        toff, tadj = _transpose(n, off, adj)
    g = HostGraph(n=n, csr_off=off, csr_dst=adj, csc_off=toff, csc_src=tadj, symmetric=symmetric, name=name)
    if weight_seed is not None:
        g.csr_w = _weights(n, off, adj, weight_seed, wmin, wmax)
        g.csc_w = g.csr_w if symmetric else _weights(n, toff, tadj, weight_seed, wmin, wmax)
    return g


def rmat_edges(scale: int, m: int, seed: int, abc=RMAT_ABC):
    src = np.empty(m, dtype=np.uint32)
    dst = np.empty(m, dtype=np.uint32)
    a, b, c = abc
    _L().gg_rmat_edges(scale, m, a, b, c, seed, _p(src), _p(dst))
    return src, dst


def rmat(scale: int, edge_factor: int = 16, seed: int = 1, symmetric: bool = False,
         abc=RMAT_ABC, weight_seed: Optional[int] = None) -> HostGraph:
    """R-MAT graph over 2^scale vertices with edge_factor * 2^scale drawn edges,
    self-loops and duplicates removed (the configurations' recipe)."""
    n = 1 << scale
    m = edge_factor * n
    src, dst = rmat_edges(scale, m, seed, abc)
    off, adj = _csr_from_edges(n, src, dst, symmetric, False, False)
    del src, dst
    if symmetric:
        toff, tadj = off, adj
    else:
        toff, tadj = _transpose(n, off, adj)
    g = HostGraph(n=n, csr_off=off, csr_dst=adj, csc_off=toff, csc_src=tadj, symmetric=symmetric,
                  name=f"rmat-s{scale}-ef{edge_factor}{'-sym' if symmetric else ''}-seed{seed}")
    if weight_seed is not None:
        g.csr_w = _weights(n, off, adj, weight_seed, 1, 255)
        g.csc_w = g.csr_w if symmetric else _weights(n, toff, tadj, weight_seed, 1, 255)
    g.meta.update(scale=scale, edge_factor=edge_factor, seed=seed, drawn_edges=m)
    return g


def symmetrise(g: HostGraph) -> HostGraph:
    """The symmetrised form of a directed graph without duplicate edges (every
    list sorted): each vertex's neighbours are the union of its out- and
    in-neighbours, itself excluded -- the graph rmat(..., symmetric=True)
    draws, built from the directed one by merging its CSR and CSC lists."""
    assert not g.symmetric and g.csr_w is None
    soff = np.zeros(g.n + 1, dtype=np.uint64)
    m = _L().gg_symmetrise(g.n, _p(g.csr_off), _p(g.csr_dst if g.m else np.zeros(1, np.int32)), _p(g.csc_off),
                           _p(g.csc_src if g.m else np.zeros(1, np.int32)), _p(soff), None)
    sadj = np.empty(max(int(m), 1), dtype=np.int32)
    _L().gg_symmetrise(g.n, _p(g.csr_off), _p(g.csr_dst if g.m else np.zeros(1, np.int32)), _p(g.csc_off),
                       _p(g.csc_src if g.m else np.zeros(1, np.int32)), _p(soff), _p(sadj))
    sadj = sadj[: int(m)]
    name = g.name + "-sym" if not g.name.endswith("-sym") else g.name
    if "-seed" in g.name:  # rmat-s26-ef16-seed5 -> rmat-s26-ef16-sym-seed5
        head, seed = g.name.rsplit("-seed", 1)
        name = f"{head}-sym-seed{seed}"
    out = HostGraph(n=g.n, csr_off=soff, csr_dst=sadj, csc_off=soff, csc_src=sadj, symmetric=True, name=name)
    out.meta.update(g.meta)
    return out


def grid_with_shortcuts(width: int = 4096, frac: float = 0.01, seed: int = 3, wmin: int = 1,
                        wmax: int = 255) -> HostGraph:
    """Undirected width x width 4-neighbour grid (row-major ids r*width+c)
    plus floor(frac * grid edges) distinct random long-range shortcuts, all
    symmetrised, with one uniform integer weight in [wmin, wmax] per
    undirected edge."""
    n = width * width
    ge = 2 * width * (width - 1)
    gsrc = np.empty(ge, dtype=np.uint32)
    gdst = np.empty(ge, dtype=np.uint32)
    k = _L().gg_grid_edges(width, width, _p(gsrc), _p(gdst))
    assert k == ge
    ns = int(math.floor(frac * ge))
    ssrc = np.empty(max(ns, 1), dtype=np.uint32)
    sdst = np.empty(max(ns, 1), dtype=np.uint32)
    if ns:
        _L().gg_grid_shortcuts(width, width, ns, seed, _p(ssrc), _p(sdst))
    src = np.concatenate([gsrc, ssrc[:ns]])
    dst = np.concatenate([gdst, sdst[:ns]])
    del gsrc, gdst
    off, adj = _csr_from_edges(n, src, dst, True, False, False)
    g = HostGraph(n=n, csr_off=off, csr_dst=adj, csc_off=off, csc_src=adj, symmetric=True,
                  name=f"grid{width}x{width}-sc{ns}-seed{seed}")
    g.csr_w = _weights(n, off, adj, seed, wmin, wmax)
    g.csc_w = g.csr_w
    g.meta.update(width=width, shortcuts=ns, seed=seed)
    return g


def rmat_small(n: int, edge_factor: int, seed: int, abc=RMAT_ABC) -> HostGraph:
    """Directed R-MAT over exactly n vertices: draws over 2^ceil(log2 n) ids,
    keeping those with both ends < n until edge_factor*n are kept, then
    self-loops and duplicates removed."""
    scale = max(1, int(math.ceil(math.log2(n))))
    want = edge_factor * n
    src = np.empty(want, dtype=np.uint32)
    dst = np.empty(want, dtype=np.uint32)
    a, b, c = abc
    _L().gg_rmat_edges_bounded(scale, n, want, a, b, c, seed, _p(src), _p(dst))
    g = from_edges(n, src, dst, symmetric=False, name=f"rmat-n{n}-ef{edge_factor}-seed{seed}")
    g.meta.update(edge_factor=edge_factor, seed=seed)
    return g


def small_graph_family(count: int = 64, lo_log2: float = 10.0, hi_log2: float = 16.0,
                       edge_factor: int = 8, seed: int = 41) -> list:
    """`count` directed R-MAT graphs with n_i = floor(2^u_i), u_i uniform in
    [lo_log2, hi_log2] (stream seed), graph i seeded with seed + i."""
    graphs = []
    for i in range(count):
        u = lo_log2 + (hi_log2 - lo_log2) * (int(_L().gg_splitmix_draw(seed, 9, i)) >> 11) / float(1 << 53)
        n = int(math.floor(2.0 ** u))
        graphs.append(rmat_small(n, edge_factor, seed + i))
    return graphs


def disjoint_union(graphs: list, name: str = "union") -> HostGraph:
    """Block-diagonal union: graph i's vertices are renumbered to start at
    the sum of the earlier graphs' vertex counts.  meta["parts"] holds the
    P+1 vertex offsets (uint32)."""
    offs = np.zeros(len(graphs) + 1, dtype=np.int64)
    for i, g in enumerate(graphs):
        offs[i + 1] = offs[i] + g.n
    eoffs = np.zeros(len(graphs) + 1, dtype=np.int64)
    for i, g in enumerate(graphs):
        eoffs[i + 1] = eoffs[i] + g.m

    def cat(attr_off, attr_adj):
        off = np.zeros(offs[-1] + 1, dtype=np.uint64)
        adj = np.empty(eoffs[-1], dtype=np.int32)
        for i, g in enumerate(graphs):
            o = getattr(g, attr_off).astype(np.int64)
            off[offs[i] + 1: offs[i + 1] + 1] = (o[1:] + eoffs[i]).astype(np.uint64)
            adj[eoffs[i]: eoffs[i + 1]] = getattr(g, attr_adj).astype(np.int64) + offs[i]
        return off, adj

    csr_off, csr_dst = cat("csr_off", "csr_dst")
    sym = all(g.symmetric for g in graphs)
    csc_off, csc_src = (csr_off, csr_dst) if sym else cat("csc_off", "csc_src")
    u = HostGraph(n=int(offs[-1]), csr_off=csr_off, csr_dst=csr_dst, csc_off=csc_off, csc_src=csc_src,
                  symmetric=sym, name=name)
    u.meta["parts"] = offs.astype(np.uint32)
    return u


def pick_sources(g: HostGraph, count: int, seed: int) -> np.ndarray:
    """`count` distinct vertices uniform among those with out-degree >= 1."""
    elig = (np.diff(g.csr_off) > 0).astype(np.uint8)
    assert int(elig.sum()) >= count
    out = np.empty(count, dtype=np.uint32)
    _L().gg_pick_sources(g.n, _p(elig), count, seed, _p(out))
    return out


# Named workloads (sizes, seeds and structure of the configurations).
def workload(name: str) -> HostGraph:
    if name == "rmat-s14-dir":
        return rmat(14, 16, seed=1, symmetric=False)
    if name == "rmat-s20-sym":
        return rmat(20, 16, seed=2, symmetric=True)
    if name == "grid4096-sc":
        return grid_with_shortcuts(4096, 0.01, seed=3)
    if name == "rmat-s22-sym":
        return rmat(22, 16, seed=4, symmetric=True)
    if name == "rmat-s26-dir":
        return rmat(26, 16, seed=5, symmetric=False)
    if name == "rmat-s26-sym":
        return symmetrise(rmat(26, 16, seed=5, symmetric=False))
    raise KeyError(name)


def workload_pair(name: str):
    """(directed, symmetrised) forms of one R-MAT draw, the symmetrised one
    merged from the directed one (one draw and sort instead of two)."""
    if name == "rmat-s26":
        d = rmat(26, 16, seed=5, symmetric=False)
        return d, symmetrise(d)
    raise KeyError(name)


def threads() -> int:
    return int(_L().gg_max_threads())
