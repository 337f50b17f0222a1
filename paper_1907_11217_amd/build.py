"""Builds libqcsim.so in-tree: host planner sources with g++, HIP sources with
hipcc for gfx950, linked by hipcc.  Run as ``python -m paper_1907_11217_amd.build``."""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libqcsim.so")
BUILD = os.path.join(HERE, "_build")

HOST_SOURCES = ["network.cpp", "order.cpp", "lower.cpp", "capi.cpp"]
HIP_SOURCES = ["kernels.hip", "runtime.hip"]
ARCH = os.environ.get("QCSIM_ARCH", "gfx950")
INCLUDES = ["-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             # No packed FP32 instructions in device code.
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-pthread", "-Wall", "-Wno-sign-compare"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError(f"build step failed: {cmd[0]} {cmd[-1]}")
    return r


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        _run(["g++", *HOST_FLAGS, *INCLUDES, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        _run(["hipcc", *HIP_FLAGS, *INCLUDES, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    tmp = OUT + ".tmp"
    _run(["hipcc", "-shared", "-fPIC", "-pthread", f"--offload-arch={ARCH}", *objs, "-o", tmp])
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
