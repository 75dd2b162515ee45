"""Host logic of the blocked in-edge layout (graph flag IPG_GRAPH_BLOCKED).

The library builds the layout on the host (csrc/blocked_layout.h) before it
copies it to the device.  `blocked_layout_check.cpp` builds it from that same
header with g++ and checks every table the kernels read against the CSC it
came from (edges as a multiset, block and chunk tiling, source order, slice
cuts, partial-sum offsets, finish groups, the XCD deal, size bounds); see
its header for the list.  The graphs span the cases the GPU tests run: one
block cut into many slices, many blocks and source windows, edge-less
blocks, hubs, a dense multigraph, the empty and one-vertex graphs, and the
symmetrised R-MAT scale 20 benchmark graph.
"""
import os
import subprocess

import numpy as np
import pytest

import graphgen
from tests.graphs_small import random_graph

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    d = tmp_path_factory.mktemp("blk")
    exe = str(d / "blocked_layout_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-Wall", "-Werror", "-I", os.path.join(ROOT, "paper_2010_08781_amd", "csrc"),
                    os.path.join(ROOT, "tests", "blocked_layout_check.cpp"), "-o", exe], check=True)
    return exe, d


def run_check(checker, n, off, src, hot=None):
    exe, d = checker
    path = str(d / "csc.bin")
    with open(path, "wb") as f:
        f.write(np.uint32(n).tobytes())
        f.write(np.uint64(len(src)).tobytes())
        f.write(np.ascontiguousarray(off, dtype=np.uint64).tobytes())
        f.write(np.ascontiguousarray(src, dtype=np.int32).tobytes())
    r = subprocess.run([exe, path] + ([str(hot)] if hot is not None else []), capture_output=True, text=True,
                       timeout=300)
    line = r.stdout.strip()
    assert r.returncode == 0 and not line.startswith("FAIL"), line or r.stderr
    return line


def stats(line):
    assert line.startswith("OK "), line
    return {k: int(v) for k, v in (t.split("=") for t in line.split()[1:])}


def check_graph(checker, hg, hot=None):
    return stats(run_check(checker, hg.n, hg.csc_off, hg.csc_src, hot))


def test_one_block_many_slices(checker):
    # N = 16384 fits one block; E = 262K edges -> 4 slices, 4 * N partial sums
    s = check_graph(checker, graphgen.workload("rmat-s14-dir"))
    assert s["blocks"] == 1 and s["slices"] == 4 and s["partial"] == 4 * 16384 and s["groups"] == 16384 // 64


@pytest.mark.parametrize("sym", [False, True])
def test_many_blocks_and_windows(checker, sym):
    s = check_graph(checker, graphgen.rmat(17, 16, seed=21, symmetric=sym))
    assert s["blocks"] > 1 and s["slices"] <= 256


def test_edge_less_blocks(checker):
    n = 90000
    rng = np.random.default_rng(6)
    hg = graphgen.from_edges(n, rng.integers(0, n, 30000), rng.integers(0, 40000, 30000))
    s = check_graph(checker, hg)
    # rows 40000.. have no in-edges: their blocks are finished by groups only
    assert s["groups"] >= (n - 40000 - 20224) // 64


def test_hubs_and_ragged_chunks(checker):
    n = 5000
    rng = np.random.default_rng(4)
    src = np.concatenate([np.arange(1, n), rng.integers(0, n, 20000), np.zeros(3000, np.int64)])
    dst = np.concatenate([np.zeros(n - 1, np.int64), rng.integers(0, n, 20000), rng.integers(1, n, 3000)])
    check_graph(checker, graphgen.from_edges(n, src, dst))


@pytest.mark.parametrize("case", ["loops_dups", "single", "no_edges", "cycle", "dense", "ragged_slices"])
def test_edge_cases(checker, case):
    if case == "loops_dups":
        hg = random_graph(333, 3000, seed=3, loops=True, dups=True)
    elif case == "single":
        hg = graphgen.from_edges(1, [], [])
    elif case == "no_edges":
        hg = graphgen.from_edges(70, [], [])
    elif case == "cycle":
        n = 1000
        hg = graphgen.from_edges(n, np.arange(n), (np.arange(n) + 1) % n)
    elif case == "dense":  # few vertices, many edges: a small block cut into many slices
        hg = random_graph(300, 400000, seed=9, loops=True, dups=True)
    else:  # a slice count that is not a multiple of the 8 XCDs
        hg = random_graph(20000, 11 * 65536 - 5, seed=12, loops=True, dups=True)
    s = check_graph(checker, hg)
    if case == "ragged_slices":
        assert s["slices"] % 8 != 0


def test_hot_first_order(checker):
    # the hot-first store relabels the vertices by in-degree; the layout of
    # such a CSC (hubs first, so the first blocks are narrow) holds the same
    # invariants
    hg = graphgen.rmat(16, 16, seed=31, symmetric=True)
    order = np.argsort(-np.diff(hg.csc_off).astype(np.int64), kind="stable")
    new_id = np.empty(hg.n, np.int64)
    new_id[order] = np.arange(hg.n)
    src = np.repeat(np.arange(hg.n), np.diff(hg.csr_off).astype(np.int64))
    rg = graphgen.from_edges(hg.n, new_id[src], new_id[hg.csr_dst], keep_self_loops=True)
    s = check_graph(checker, rg)
    assert s["blocks"] > 1


def test_many_row_blocks_cut_dense_blocks(checker):
    # 8.4M vertices: more row-capped blocks (415) than slices (256), so the
    # blocks run in rounds; the dense rows form narrow blocks (at most twice
    # the mean edges of a row-capped block) and the costliest blocks are cut
    # into slices with partial sums
    hg = graphgen.rmat(23, 4, seed=5)
    s = check_graph(checker, hg)
    assert s["blocks"] > 415 and s["slices"] > s["blocks"] - 2 and s["partial"] > 0


def test_rejects_malformed_csc(checker):
    assert run_check(checker, 3, [0, 1, 2, 2], [0, 5]).startswith("ERR CSC source id")
    assert run_check(checker, 3, [0, 2, 1, 2], [0, 1]).startswith("ERR offsets decreasing")
    assert run_check(checker, 3, [1, 1, 2, 2], [0, 1]).startswith("ERR offsets")
    assert run_check(checker, 2, [0, 1, 1], [-1]).startswith("ERR CSC source id")


def test_benchmark_graph_rmat_s20_symmetrised(checker):
    s = check_graph(checker, graphgen.workload("rmat-s20-sym"))
    assert s["slices"] == 256


# ------------------------------------------------- binned cold sources ----

@pytest.mark.parametrize("sym", [False, True])
def test_binned_rmat_s17(checker, sym):
    # N = 131072: hot sources [0, 65536), cold scatter windows 4..7
    hg = graphgen.rmat(17, 16, seed=21, symmetric=sym)
    s = check_graph(checker, hg, hot=65536)
    assert s["hot"] == 65536 and s["slots"] > 0 and s["runs"] > 0 and s["slots"] % 8 == 0
    # a hot count past N: no binning
    assert check_graph(checker, hg, hot=1 << 20)["hot"] == 0


def test_binned_rounds_hot_up_to_windows(checker):
    hg = graphgen.rmat(18, 8, seed=3)
    assert check_graph(checker, hg, hot=1000)["hot"] == 65536
    assert check_graph(checker, hg, hot=65537)["hot"] == 131072


def test_binned_multigraph_hubs_and_empty_ranges(checker):
    # loops, duplicate edges (two edges from one source to one row share a
    # slot), a hub destination, a cold source hitting many blocks, and a
    # range of rows without in-edges
    n = 300000
    rng = np.random.default_rng(8)
    src = np.concatenate([rng.integers(0, n, 400000), np.full(50000, 250001), rng.integers(0, n, 30000)])
    dst = np.concatenate([rng.integers(0, 200000, 400000), rng.integers(0, 200000, 50000), np.zeros(30000, np.int64)])
    hg = graphgen.from_edges(n, src, dst, keep_self_loops=True, keep_duplicates=True)
    s = check_graph(checker, hg, hot=65536)
    assert s["hot"] == 65536 and s["slots"] >= 1


def test_binned_every_source_cold_window(checker):
    # all edges from cold sources in one scatter window
    n = 140000
    rng = np.random.default_rng(2)
    hg = graphgen.from_edges(n, rng.integers(131072, 131072 + 16384, 60000), rng.integers(0, n, 60000))
    s = check_graph(checker, hg, hot=65536)
    assert s["hot"] == 65536


@pytest.mark.slow
def test_binned_rmat_s20(checker):
    hg = graphgen.rmat(20, 16, seed=5)
    s = check_graph(checker, hg, hot=1 << 18)
    assert s["hot"] == 1 << 18


BIN_PLANTS = {
    "slot offset off by one": ("packed[i] |= d << 16;", "packed[i] |= (d + 1) << 16;"),
    "group entry past its run": ("while (r + 1 < rstart[w + 1] && wruns[r + 1].flat <= j) ++r;",
                                 "while (r + 1 < rstart[w + 1] && wruns[r + 1].flat < j) ++r;"),
    "source offset truncated": ("slot_src[r.dst + j] & ((1u << kBinWinBits) - 1)",
                                "slot_src[r.dst + j] & ((1u << (kBinWinBits - 1)) - 1)"),
    "cold chunk base off by one": ("chunks.push_back(BlkChunk{at, base, static_cast<uint16_t>(m), 1});",
                                   "chunks.push_back(BlkChunk{at, base + 1, static_cast<uint16_t>(m), 1});"),
    "runs not padded": ("if (!runs.empty() && runs.back().len % kBinPad) {  // pad the run this one follows",
                        "if (false) {"),
}


@pytest.mark.parametrize("plant", sorted(BIN_PLANTS))
def test_checker_catches_planted_binning_mistakes(tmp_path, plant):
    # the same build with one mistake planted in a copy of the header: the
    # checker must reject its tables
    old, new = BIN_PLANTS[plant]
    src_dir = os.path.join(ROOT, "paper_2010_08781_amd", "csrc")
    text = open(os.path.join(src_dir, "blocked_layout.h")).read()
    assert text.count(old) == 1, plant
    (tmp_path / "blocked_layout.h").write_text(text.replace(old, new))
    exe = str(tmp_path / "check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", str(tmp_path), os.path.join(ROOT, "tests", "blocked_layout_check.cpp"),
                    "-o", exe], check=True)
    hg = random_graph(200000, 600000, seed=12, loops=True, dups=True)
    path = str(tmp_path / "csc.bin")
    with open(path, "wb") as f:
        f.write(np.uint32(hg.n).tobytes())
        f.write(np.uint64(hg.m).tobytes())
        f.write(np.ascontiguousarray(hg.csc_off, dtype=np.uint64).tobytes())
        f.write(np.ascontiguousarray(hg.csc_src, dtype=np.int32).tobytes())
    r = subprocess.run([exe, path, "65536"], capture_output=True, text=True, timeout=300)
    out = r.stdout.strip()
    assert out.startswith("FAIL") or out.startswith("ERR"), f"planted mistake passed: {out!r} rc={r.returncode}"


@pytest.mark.parametrize("hot", [None, 65536])
def test_several_rounds_costliest_first(checker, hot):
    # more row-capped blocks than one wave of slices: the launch order is by
    # descending cost (the checker recomputes each slice's cost)
    n = 6_000_000
    rng = np.random.default_rng(13)
    src = np.concatenate([rng.integers(0, n, 1_500_000), rng.integers(0, 1000, 500_000)])
    dst = np.concatenate([rng.integers(0, n, 1_500_000), rng.integers(0, 40_000, 500_000)])
    hg = graphgen.from_edges(n, src, dst)
    s = check_graph(checker, hg, hot=hot)
    assert s["slices"] > 256
