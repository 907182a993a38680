"""Build ``libimexlb.so`` (HIP for gfx950) in-tree with hipcc.

Run ``python -m paper_1909_08390_amd.build`` or call :func:`build`.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libimexlb.so")

SOURCES = [os.path.join(CSRC, "imexlb.cpp"), os.path.join(CSRC, "batch.cpp"),
           os.path.join(CSRC, "kernels.hip"), os.path.join(CSRC, "adjoint.hip"),
           os.path.join(CSRC, "probe.hip"), os.path.join(CSRC, "reduce.hip"),
           os.path.join(CSRC, "noalloc.hip")]

# Packed FP32 instructions are disabled for all device code (the compiler
# would otherwise form v_pk_* ops from float code).
HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, "-I", INCLUDE, "-I", CSRC, *SOURCES, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd, cwd=PKG)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
