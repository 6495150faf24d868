"""Build libfse.so (HIP kernels for gfx950 + C++ host runtime) in-tree.

Usage: python -m paper_2207_00233_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfse.so")
ARCH = os.environ.get("FSE_OFFLOAD_ARCH", "gfx950")

SOURCES = ["fse_kernels.hip", "fse_runtime.cpp", "fse_sched.cpp", "fse_serve.cpp",
           "fse_volume.hip", "fse_volume.cpp", "fse_peaks.hip"]

# Packed FP32 instructions are switched off for the device code.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    return "hipcc"


def build(verbose: bool = False, extra=None) -> str:
    """Compile every source into ``libfse.so`` next to this file."""
    objs = []
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(bdir, src + ".o")
        cmd = [hipcc(), "-c", "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
               "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-Wall",
               "-Wno-unused-command-line-argument"]
        if src.endswith(".hip"):
            cmd += ["-x", "hip"] + DEVICE_FLAGS
        cmd += list(extra or []) + ["-o", obj, path]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs + ["-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
