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


def test_struct_layouts_match_header(tmp_path):
    """The ctypes structures against the C compiler's layout of the header's structures."""
    import shutil
    import subprocess
    from paper_2510_23215_amd import scsf
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    structs = {"scsf_operator": scsf.Operator, "scsf_params": scsf.Params,
               "scsf_stats": scsf.Stats, "scsf_profile": scsf.Profile}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "scsf.h"', 'int main(void) {']
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
