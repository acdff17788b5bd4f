"""Build the HIP library libspchol.so in-tree for gfx950 with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libspchol.so")
SOURCES = ["symbolic.cpp", "ordering.cpp", "capi.cpp", "kernels.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    "-munsafe-fp-atomics",
    # packed FP32 instructions stay off in all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


TASKLIB = os.path.join(HERE, "libtaskchol.so")
# the host task-parallel CPU baseline: plain C++ with OpenMP, for any x86-64
# with AVX2 and FMA (built once, run on the host of the GPU machine)
TASK_FLAGS = ["-O3", "-std=c++17", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared", "-Wall"]


def build_taskchol(verbose: bool = False) -> str:
    tmp = TASKLIB + f".tmp{os.getpid()}"
    cmd = ["g++", *TASK_FLAGS, os.path.join(CSRC, "taskchol.cpp"), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, TASKLIB)
    return TASKLIB


def build(verbose: bool = False) -> str:
    """Compile every source and link libspchol.so (and the host baseline
    libtaskchol.so); returns the path of libspchol.so."""
    build_taskchol(verbose)
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
