"""Host-side checks of the C-ABI library (no GPU compute): it loads, and it
exports every function include/ccham.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ccham.h")
LIB = os.path.join(ROOT, "paper_1709_03005_amd", "libccham.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cch_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ["cch_create", "cch_destroy", "cch_set_orbitals", "cch_set_integrals",
              "cch_add_target_symmetry", "cch_set_l2", "cch_plan", "cch_build", "cch_get_matrix",
              "cch_get_labels", "cch_davidson"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    lib = ctypes.CDLL(LIB)
    for n in declared():
        assert hasattr(lib, n), n


def test_binding_lists_the_same_symbols():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    import paper_1709_03005_amd as cc
    assert sorted(cc.EXPORTS) == declared()
    assert "gfx950" in cc.version()


def test_version_and_error_without_context():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    lib = ctypes.CDLL(LIB)
    lib.cch_version.restype = ctypes.c_char_p
    lib.cch_destroy.argtypes = [ctypes.c_void_p]
    assert lib.cch_version().startswith(b"ccham")
    assert lib.cch_destroy(None) == 0
