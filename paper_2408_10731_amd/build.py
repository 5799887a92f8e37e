"""Builds the gfx950 HIP library libtrajam.so in-tree with hipcc.

Every HIP translation unit is compiled with packed-FP32 instructions disabled
(`-Xclang -target-feature -Xclang -packed-fp32-ops`); the obstacle loop is plain
scalar float/double code, so nothing is lost by keeping the compiler from pairing it.
"""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtrajam.so")
SOURCES = ["am_kernels.hip", "polar_kernels.hip", "cem_kernels.hip", "mlp_kernels.hip", "mpc_kernels.hip",
           "heading_kernels.hip", "trajam_api.cpp", "mlp_api.cpp", "heading_api.cpp"]
ARCH = os.environ.get("TRAJAM_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["-O3", "-fPIC", "-std=c++17", "-mcode-object-version=5", "-Wall", "-Wno-unused-function",
          "-Wno-unused-variable", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False) -> str:
    """Compile every source (always; build products are not trusted) and link."""
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)

    def compile_one(src):
        obj = os.path.join(bdir, src + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [HIPCC, f"--offload-arch={ARCH}", *COMMON, *lang, "-c",
               os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        return obj

    # the sources compile independently: one process each
    with concurrent.futures.ThreadPoolExecutor(max_workers=len(SOURCES)) as pool:
        objs = list(pool.map(compile_one, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
