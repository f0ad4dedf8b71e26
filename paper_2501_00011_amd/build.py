"""Build libmcchem.so in-tree with hipcc for gfx950.

Every source is compiled to its own object in parallel (each carries its own
device code and launches only its own kernels), then the objects are linked.

Usage: python -m paper_2501_00011_amd.build   (or build() from Python).
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB_PATH = os.path.join(HERE, "libmcchem.so")
OBJ_DIR = os.path.join(ROOT, "_build", "mcchem")
SOURCES = ["csrc/api.hip", "csrc/kernels_fj.hip", "csrc/kernels_solve.hip", "csrc/mech_compile.cpp",
           "csrc/mech_emulate.cpp", "csrc/fj_codegen.cpp", "csrc/kernels_paper.hip"]
ARCH = os.environ.get("MCC_OFFLOAD_ARCH", "gfx950")

# Packed FP32 instructions stay off: the library computes in FP64, and packed
# FP32 forms are not needed anywhere.
HIP_FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-result"]


def build(verbose: bool = False, extra=()) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ_DIR, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include")]

    def compile_one(src):
        obj = os.path.join(OBJ_DIR, os.path.basename(src) + ".o")
        cmd = [hipcc, *HIP_FLAGS, *extra, *inc, "-c", "-o", obj, os.path.join(HERE, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        return obj

    jobs = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(jobs) as pool:
        objs = list(pool.map(compile_one, SOURCES))
    tmp = LIB_PATH + ".tmp"
    cmd = [hipcc, *HIP_FLAGS, *extra, "-shared", "-o", tmp, *objs, "-lhiprtc"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
