"""Build the HIP library (liblattice_tdse.so) for gfx950 with hipcc.

The library exports exactly the C-ABI declared in include/lattice_tdse.h.
Packed FP32 instructions are disabled for all device code.  Each source is
compiled to its own object in parallel (no device code crosses translation
units), then the objects are linked into the shared library.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "_lib")
OBJDIR = os.path.join(HERE, "_build")
LIB = os.path.join(LIBDIR, "liblattice_tdse.so")
SOURCES = ["planner.cpp", "capi.cpp", "timing.cpp", "kernels.hip", "kernels_fast.hip", "noalloc.hip"]
HEADERS = ["lt_internal.h", os.path.join("..", "..", "include", "lattice_tdse.h")]
ARCH = os.environ.get("LT_OFFLOAD_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include")]


def compile_command(src: str, obj: str):
    return ["hipcc"] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]


def link_command(objs, out: str):
    return ["hipcc", f"--offload-arch={ARCH}", "-fPIC", "-shared"] + list(objs) + ["-o", out]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    return res.returncode, res.stdout + res.stderr


def build(verbose: bool = False) -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    os.makedirs(OBJDIR, exist_ok=True)
    tag = f".{os.getpid()}.o"
    objs = [os.path.join(OBJDIR, os.path.splitext(s)[0] + tag) for s in SOURCES]
    jobs = int(os.environ.get("LT_BUILD_JOBS", str(min(len(SOURCES), os.cpu_count() or 1))))
    try:
        with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
            results = list(ex.map(lambda so: _run(compile_command(*so), verbose), zip(SOURCES, objs)))
        for (rc, out), src in zip(results, SOURCES):
            if rc != 0:
                sys.stderr.write(out)
                raise RuntimeError(f"hipcc failed to compile {src}")
        tmp = LIB + f".tmp{os.getpid()}"
        rc, out = _run(link_command(objs, tmp), verbose)
        if rc != 0:
            sys.stderr.write(out)
            raise RuntimeError("hipcc failed to link liblattice_tdse.so")
        os.replace(tmp, LIB)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
