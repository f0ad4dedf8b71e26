"""Build libmcchem.so in-tree with hipcc for gfx950.

Usage: python -m paper_2501_00011_amd.build   (or build() from Python).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB_PATH = os.path.join(HERE, "libmcchem.so")
SOURCES = ["csrc/api.hip", "csrc/kernels_fj.hip", "csrc/kernels_solve.hip", "csrc/mech_compile.cpp",
           "csrc/mech_emulate.cpp", "csrc/fj_codegen.cpp", "csrc/kernels_paper.hip"]
ARCH = os.environ.get("MCC_OFFLOAD_ARCH", "gfx950")

# Packed FP32 instructions stay off: the library computes in FP64, and packed
# FP32 forms are not needed anywhere.
HIP_FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-shared",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-result"]


def build(verbose: bool = False, extra=()) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    tmp = LIB_PATH + ".tmp"
    cmd = [hipcc, *HIP_FLAGS, *extra, "-I", os.path.join(ROOT, "include"), "-o", tmp, *srcs, "-lhiprtc"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
