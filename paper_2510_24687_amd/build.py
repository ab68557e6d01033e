"""Build the in-tree HIP library ``libpat.so`` for gfx950.

Compiles the kernels and the host plan builder with hipcc (packed-FP32
instructions disabled) into ``paper_2510_24687_amd/libpat.so``.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libpat.so")
SOURCES = [os.path.join(CSRC, "pat_kernels.hip"), os.path.join(CSRC, "pat_solvers.hip"),
           os.path.join(CSRC, "pat_lpd.hip"), os.path.join(CSRC, "pat_unet.hip"),
           os.path.join(CSRC, "pat_plan.cpp")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# code-generation flags shared by every source: packed FP32 arithmetic is
# switched off in the device code
FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + ["-fPIC", "-shared", "-Wall", "-Wno-unused-result", "-o", tmp] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
