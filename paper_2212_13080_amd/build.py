"""Build libeqfmm.so for gfx950 with hipcc (in-tree, next to this file).

Each source is compiled to its own object in parallel, then the objects are
linked into the shared library (no device code crosses translation units).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["csrc/plan.cpp", "csrc/kernels.hip", "csrc/m2l.hip", "csrc/near.hip"]
LIB = os.path.join(HERE, "libeqfmm.so")
OBJDIR = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed FP32 arithmetic is disabled on purpose: the compiler is not allowed
# to fuse float pairs into packed instructions.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]


def build_library(verbose: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    objs, procs = [], []
    for s in SOURCES:
        obj = os.path.join(OBJDIR, os.path.basename(s) + ".o")
        cmd = [HIPCC] + FLAGS + ["-c", "-o", obj, os.path.join(HERE, s)]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd)))
        objs.append(obj)
    failed = [cmd for cmd, p in procs if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build_library(verbose="-v" in sys.argv)
