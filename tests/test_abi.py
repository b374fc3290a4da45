"""The C-ABI library loads and exports every function that include/qhap.h declares
(no compute call: this runs without a GPU)."""
import ctypes
import os
import re

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
