"""Build the HIP library (liblattice_tdse.so) for gfx950 with hipcc.

The library exports exactly the C-ABI declared in include/lattice_tdse.h.
Packed FP32 instructions are disabled for all device code.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "_lib")
LIB = os.path.join(LIBDIR, "liblattice_tdse.so")
SOURCES = ["planner.cpp", "capi.cpp", "timing.cpp", "kernels.hip", "kernels_fast.hip"]
HEADERS = ["lt_internal.h", os.path.join("..", "..", "include", "lattice_tdse.h")]
ARCH = os.environ.get("LT_OFFLOAD_ARCH", "gfx950")


def command(out: str):
    return (["hipcc", "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-shared",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument",
             "-I", os.path.join(ROOT, "include")]
            + [os.path.join(CSRC, s) for s in SOURCES] + ["-o", out])


def build(verbose: bool = False) -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed to build liblattice_tdse.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
