"""Hypothesis strategies for small random graphs (inputs only; no method arithmetic)."""
import numpy as np
from hypothesis import strategies as st

import graphgen


@st.composite
def small_graphs(draw, max_n=48, max_m=240, weighted=None):
    """A small graph from a random edge list: any n >= 1, self-loops and
    duplicate edges kept or dropped, directed or symmetrised, optionally
    weighted (weights in [1, 255])."""
    n = draw(st.integers(1, max_n))
    m = draw(st.integers(0, max_m))
    src = draw(st.lists(st.integers(0, n - 1), min_size=m, max_size=m))
    dst = draw(st.lists(st.integers(0, n - 1), min_size=m, max_size=m))
    sym = draw(st.booleans())
    loops = draw(st.booleans())
    dups = draw(st.booleans())
    w = draw(st.booleans()) if weighted is None else weighted
    seed = draw(st.integers(0, 2**31 - 1))
    return graphgen.from_edges(n, np.array(src, dtype=np.int64), np.array(dst, dtype=np.int64), symmetric=sym,
                               keep_self_loops=loops, keep_duplicates=dups,
                               weight_seed=seed if w else None, name=f"hyp-n{n}-m{m}")
