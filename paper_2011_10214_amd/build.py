"""Builds the HIP library ``libpic.so`` (gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpic.so")
SOURCES = [os.path.join(CSRC, "pic_kernels.hip"), os.path.join(CSRC, "pic_field.hip"),
           os.path.join(CSRC, "pic_capi.cpp")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # no fused multiply-add unless written as fma: results follow the
    # expression order of the method's definition
    "-ffp-contract=off",
    # no packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # hardware float atomics on (coarse-grained) device memory
    "-munsafe-fp-atomics",
    "-Wno-unused-command-line-argument",
]
# roctx ranges around the library's calls (for profilers)
LIBS = ["-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]


def build(verbose: bool = False) -> str:
    """Compile every source into libpic.so (always recompiles)."""
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, *SOURCES, *LIBS, "-o", tmp]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
