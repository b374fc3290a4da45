"""The C-ABI library loads and exports every function that include/qhap.h declares
(no compute call: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

import paper_2603_25762_amd as qh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "qhap.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qh_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("qh_build_graph", "qh_bsb_solve", "qh_bsb_solve_batched", "qh_phase"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(qh.lib_path)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_version_string():
    assert qh.version().startswith("qhap-gfx950")


def test_adaptive_schedule_follows_the_paper():
    """SNP-based settings adapted to graph size (Tables 1 and 2, footnotes), from the C entry
    point (host only): 500 iterations below 5,000 vertices, 1,000 from there on, 100 samples
    (run as 128 replicas, the replica counts being 16, 32 or multiples of 64) and at most 15
    refinement rounds."""
    for n, steps in ((0, 500), (1, 500), (4999, 500), (5000, 1000), (120_000, 1000)):
        a = qh.adaptive_schedule(n)
        assert a["steps"] == steps and a["samples"] == 100 and a["max_rounds"] == 15
        assert a["replicas"] >= a["samples"] and a["replicas"] % 64 == 0 and a["size"] == n
    with pytest.raises(qh.QhapError) as e:
        qh.adaptive_schedule(-1)
    assert e.value.status == qh.Status.EINVAL


def test_build_graphs_validates_on_the_host():
    """qh_build_graphs rejects a negative count and a thread count outside 0..64 before any
    device call, and an empty batch is a no-op; the binding returns no graphs for no specs."""
    lib = qh.load()
    assert lib.qh_build_graphs(-1, None, None, None, None, 0, None) == qh.Status.EINVAL
    assert lib.qh_build_graphs(1, None, None, None, None, 65, None) == qh.Status.EINVAL
    assert lib.qh_build_graphs(1, None, None, None, None, -1, None) == qh.Status.EINVAL
    assert lib.qh_build_graphs(0, None, None, None, None, 0, None) == qh.Status.OK
    assert qh.build_graphs([]) == []


def test_phase_batched_validates_on_the_host():
    """qh_phase_batched rejects a negative graph count and null arrays before any device
    call; an empty list is a no-op."""
    lib = qh.load()
    assert lib.qh_phase_batched(None, -1, None, None, None, None) == qh.Status.EINVAL
    assert lib.qh_phase_batched(None, 0, None, None, None, None) == qh.Status.OK
    assert lib.qh_phase_batched(None, 2, None, None, None, None) == qh.Status.EINVAL


def test_release_cached_memory_without_cached_blocks():
    """With nothing cached the release makes no device call and reports zero bytes."""
    assert qh.release_cached_memory() == 0
