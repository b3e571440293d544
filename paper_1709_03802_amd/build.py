"""Compile the gfx950 HIP library (libdartray.so) in-tree with hipcc."""

from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libdartray.so")
CEIL_LIB = os.path.join(PKG, "libdrceil.so")
SOURCES = [os.path.join(CSRC, "dartray.hip")]
CEIL_SOURCES = [os.path.join(CSRC, "ceilings.hip")]
HEADERS = [os.path.join(CSRC, "dr_internal.h"), os.path.join(INCLUDE, "dartray.h")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed-FP32 instructions anywhere in this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def hipcc() -> str:
    for cand in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.isabs(cand) and os.path.exists(cand):
            return cand
    return "hipcc"


def build(verbose: bool = False) -> str:
    """Always recompiles (the caller decides when to build)."""
    for lib, srcs in ((LIB, SOURCES), (CEIL_LIB, CEIL_SOURCES)):
        tmp = lib + ".tmp"
        cmd = [hipcc(), *HIPCC_FLAGS, "-I", INCLUDE, "-I", CSRC, "-o", tmp, *srcs]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        os.replace(tmp, lib)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
