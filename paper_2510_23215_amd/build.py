"""Build libscsf.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_2510_23215_amd.build        # or paper_2510_23215_amd.build.build()
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libscsf.so")
ARCH = "gfx950"

SOURCES = ["spmm.hip", "gemm.hip", "dense.hip", "tridiag.hip", "misc.hip", "sort.hip", "diag.hip",
           "cnn.hip", "solver.cpp"]

# Packed FP32 instructions are disabled for all device code (the compiler would otherwise
# form v_pk_* FP32 operations from scalar float code).
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-result"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every source to an object in csrc/_build, then link libscsf.so.  Always
    recompiles (the check that the HIP code builds)."""
    out_dir = os.path.join(CSRC, "_build")
    os.makedirs(out_dir, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(out_dir, src.replace(".", "_") + ".o")
        objs.append(obj)
        lang = ["-x", "hip"]
        cmd = [hipcc(), *lang, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((src, cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                                 stderr=subprocess.STDOUT, text=True)))
        if len(procs) >= jobs:
            _drain(procs[:1], verbose)
            procs = procs[1:]
    _drain(procs, verbose)
    tmp = LIB + ".tmp"
    link = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(link, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def _drain(procs, verbose):
    for src, cmd, p in procs:
        out, _ = p.communicate()
        lines = [l for l in (out or "").splitlines() if "packed-fp32-ops" not in l]
        if p.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n" + "\n".join(lines))
        if verbose and lines:
            print("\n".join(lines))


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
