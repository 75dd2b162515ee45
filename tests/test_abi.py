"""The C-ABI library loads and exports every symbol the public header declares.

Only host-side logic is exercised here (size queries and argument checks that
return before any device call), so this runs without a GPU.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ipregel.h")
LIB = os.path.join(ROOT, "paper_2010_08781_amd", "libipregel.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ipg_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libipregel.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_interface():
    names = declared_functions()
    for n in ("ipg_graph_create", "ipg_run", "ipg_read_values", "ipg_graph_destroy", "ipg_last_error",
              "ipg_graph_workspace_bytes", "ipg_run_workspace_bytes"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_workspace_sizes_scale(lib):
    lib.ipg_run_workspace_bytes.restype = ctypes.c_size_t
    lib.ipg_run_workspace_bytes.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int]
    lib.ipg_graph_workspace_bytes.restype = ctypes.c_size_t
    lib.ipg_graph_workspace_bytes.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32]
    n, e = 1 << 20, 1 << 25
    pr = lib.ipg_run_workspace_bytes(n, e, 0)
    cc = lib.ipg_run_workspace_bytes(n, e, 1)
    assert pr >= 3 * 8 * n and cc >= 5 * 4 * n
    assert pr % 256 == 0 and cc % 256 == 0
    g = lib.ipg_graph_workspace_bytes(n, e, 0)
    # out-degrees plus the pull tiling tables and work items: a 24-byte item
    # per 256-edge row group, per 64 rows and per long-row chunk, so well
    # under half a byte per edge
    assert 4 * n <= g < 4 * n + (3 * e) // 8 + n // 2 + 4096


def test_null_arguments_rejected_before_any_device_call(lib):
    import paper_2010_08781_amd as ipg

    L = ipg.lib()
    h = ctypes.c_void_p()
    assert L.ipg_graph_create(None, None, 0, None, ctypes.byref(h)) == ipg.EINVAL
    assert h.value is None
    assert "desc" in ipg.last_error()
    assert L.ipg_run(None, 0, 0, 10, None, None, 0, None, None) == ipg.EINVAL
    assert L.ipg_read_values(None, None, 0, 0, None) == ipg.EINVAL
    d = ipg._Desc(0, 0, None, None, None, None, None, None, 0)
    assert L.ipg_graph_create(ctypes.byref(d), None, 0, None, ctypes.byref(h)) == ipg.EINVAL
    d = ipg._Desc(4, 0, 64, None, 64, None, None, None, 0)
    assert L.ipg_graph_create(ctypes.byref(d), None, 0, None, ctypes.byref(h)) == ipg.EWORKSPACE


def test_binding_refuses_missing_library(monkeypatch, tmp_path):
    import paper_2010_08781_amd as ipg

    monkeypatch.setattr(ipg, "_lib", None)
    monkeypatch.setattr(ipg, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(ImportError):
        ipg.lib()


def test_footprint_report_adds_up(lib):
    import paper_2010_08781_amd as ipg

    n, m = 1 << 20, 31 << 20
    f = ipg.footprint(n, m, symmetric=True, rename=False)
    assert f["graph_arrays"]["csc"] == 0 and f["graph_arrays"]["csr"] == 8 * (n + 1) + 4 * m
    d = ipg.footprint(n, m, symmetric=False, weighted=True)
    assert d["graph_arrays"]["csc"] == d["graph_arrays"]["csr"] and d["graph_arrays"]["weights"] == 8 * m
    for k, v in f["total"].items():
        assert v == sum(f["graph_arrays"].values()) + f["graph_workspace"] + f["run_workspace"][k]
    # the run state is a few words per vertex; the graph is ids plus offsets
    assert f["bytes_per_vertex_run"]["pagerank"] < 48 and f["bytes_per_vertex_run"]["cc"] < 40
    # batched SSSP: 256-bit visited and receive rows plus a 16-superstep ring of level masks
    assert f["bytes_per_vertex_run"]["multi_sssp"] < (16 + 2) * 32 + 64
    assert 4.0 <= f["bytes_per_edge"]["cc"] < 6.5
    # the hot-first copy of the sources adds 4 bytes per edge and 4 per vertex
    r = ipg.footprint(n, m, symmetric=True, rename=True)
    assert r["graph_workspace"] - f["graph_workspace"] >= 4 * m + 4 * n


def test_blocked_tables_per_store(lib):
    # A hot-first blocked store keeps a second blocked table, on the caller's
    # CSC, for CC/SSSP -- unless it is symmetric: CC and SSSP then run under
    # the new names on the hot-first table, so the symmetric store is one
    # table (about 4E bytes) smaller than the directed one of the same size.
    import paper_2010_08781_amd as ipg

    n, m = 1 << 20, 31 << 20
    for binned in (False, True):
        sym = ipg.footprint(n, m, symmetric=True, rename=True, blocked=True, binned=binned)["graph_workspace"]
        dirg = ipg.footprint(n, m, symmetric=False, rename=True, blocked=True, binned=binned)["graph_workspace"]
        plain = ipg.footprint(n, m, symmetric=True, rename=True)["graph_workspace"]
        assert dirg - sym >= 4 * m, binned
        assert sym - plain >= 4 * m, binned  # the one table it keeps
    # the renaming itself: ids, both directions, by-name out-degrees and offsets
    base = ipg.footprint(n, m, symmetric=True, rename=False)["graph_workspace"]
    assert ipg.footprint(n, m, symmetric=True, rename=True)["graph_workspace"] - base >= 4 * m + 20 * n
