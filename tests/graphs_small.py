"""Small hand-made and random test graphs (inputs only; no method arithmetic)."""
import numpy as np

import graphgen


def directed_cycle(n):
    src = np.arange(n)
    return graphgen.from_edges(n, src, (src + 1) % n, name=f"cycle{n}")


def complete_digraph(n):
    s, d = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    mask = s != d
    return graphgen.from_edges(n, s[mask], d[mask], name=f"K{n}")


def path(n, directed=False):
    src = np.arange(n - 1)
    return graphgen.from_edges(n, src, src + 1, symmetric=not directed, name=f"path{n}")


def random_graph(n, m, seed, symmetric=False, loops=False, dups=False, weight_seed=None):
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n, size=m)
    dst = rng.integers(0, n, size=m)
    return graphgen.from_edges(n, src, dst, symmetric=symmetric, keep_self_loops=loops,
                               keep_duplicates=dups, weight_seed=weight_seed, name=f"rand{n}x{m}s{seed}")


def strongly_connected_random(n, extra, seed):
    """A cycle through all vertices plus random chords: strongly connected, no dangling vertex."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    src = list(perm)
    dst = list(np.roll(perm, -1))
    src += list(rng.integers(0, n, size=extra))
    dst += list(rng.integers(0, n, size=extra))
    return graphgen.from_edges(n, np.array(src), np.array(dst), name=f"scc{n}")


def edge_arrays(g):
    """(src, dst) arrays of the CSR, in CSR order."""
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.csr_off).astype(np.int64))
    return src, g.csr_dst.astype(np.int64)
