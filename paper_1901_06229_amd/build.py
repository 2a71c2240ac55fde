"""Build the HIP library libdock.so for gfx950 (in-tree, no JIT cache)."""
from __future__ import annotations

import os
import shutil
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB_PATH = os.path.join(PKG, "libdock.so")

SOURCES = ["sweep_kernels.hip", "sweep_pruned.hip", "sweep_group.hip", "align.hip", "learned.hip", "mlp.hip", "mlp_abi.hip",
           "probe.hip", "dock_abi.hip", "hybrid.hip"]
# host-only C++ (the hybrid path's CPU sweep), compiled by the host compiler
HOST_SOURCES = ["cpu_sweep.cpp"]
HOST_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-mavx2", "-mfma", "-ffp-contract=off"]

HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def cxx() -> str:
    for c in (os.environ.get("CXX"), shutil.which("g++")):
        if c and shutil.which(c):
            return c
    raise RuntimeError("g++ not found")


def build(verbose: bool = False, out: str = LIB_PATH, defines=()) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = out + ".tmp"
    objs = []
    for s in HOST_SOURCES:
        obj = out + "." + os.path.splitext(s)[0] + ".o"
        cmd = [cxx(), *HOST_FLAGS, *[f"-D{d}" for d in defines], "-I", INCLUDE, "-I", CSRC, "-c",
               os.path.join(CSRC, s), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    cmd = [hipcc(), *HIP_FLAGS, *[f"-D{d}" for d in defines], "-I", INCLUDE, "-I", CSRC, *srcs,
           "-x", "none", *objs, "-lpthread", "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    for obj in objs:
        os.remove(obj)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
