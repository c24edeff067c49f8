"""The C-ABI library loads and exports every entry point its header declares (no GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "scsf.h")
LIB = os.path.join(ROOT, "paper_2510_23215_amd", "libscsf.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(scsf_[a-z_]+)\s*\(", text)))


def test_header_declares_the_hot_path():
    names = declared()
    for must in ["scsf_create", "scsf_destroy", "scsf_spmm", "scsf_filter", "scsf_orthonormalize",
                 "scsf_rayleigh_ritz", "scsf_bounds", "scsf_features", "scsf_sort", "scsf_solve",
                 "scsf_solve_sequence"]:
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libscsf.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared():
        assert hasattr(lib, name), name
    lib.scsf_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.scsf_version()
    lib.scsf_status_string.restype = ctypes.c_char_p
    assert lib.scsf_status_string(-3) == b"not converged within max_iter"


def test_struct_layouts_match_header():
    from paper_2510_23215_amd import scsf
    assert ctypes.sizeof(scsf.Operator) == 4 + 4 + 8 + 7 * 8 + 8
    assert ctypes.sizeof(scsf.Params) == 7 * 4 + 4 + 8 + 8
    assert ctypes.sizeof(scsf.Stats) == 6 * 4 + 8 + 8 + 8
