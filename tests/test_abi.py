"""The C-ABI library loads on a machine without a GPU and exports every
function that include/bnos.h declares (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "bnos.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(bnos_[a-z_0-9]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["bnos_build_score_table", "bnos_score_orders", "bnos_score_order", "bnos_table_free",
                 "bnos_counts", "bnos_table_export", "bnos_last_error"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    lib_path = os.path.join(ROOT, "paper_1210_5128_amd", "libbnos.so")
    if not os.path.exists(lib_path):
        pytest.fail("libbnos.so is not built")
    lib = ctypes.CDLL(lib_path)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_wraps_every_declared_symbol():
    from paper_1210_5128_amd import bnos
    assert sorted(bnos.exported_symbols()) == declared_functions()
    assert bnos.version() == 100
