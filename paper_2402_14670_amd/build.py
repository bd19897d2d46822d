"""Builds the HIP library liblf_hip.so in-tree for gfx950.

Floating-point flags are part of the method's contract: binary32 with no
contraction into FMA (-ffp-contract=off), no fast-math, correctly rounded
division and square root, denormals kept, and no packed-FP32 instructions.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblf_hip.so")
SOURCES = [os.path.join(CSRC, "lf_api.cpp"), os.path.join(CSRC, "lf_serve.cpp"), os.path.join(CSRC, "lf_kernels.hip")]
HEADERS = [os.path.join(CSRC, "lf_internal.h"), os.path.join(ROOT, "include", "lf.h")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("LF_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared", "-pthread",
    "-ffp-contract=off", "-fno-fast-math", "-fno-gpu-flush-denormals-to-zero",
    "-fhip-fp32-correctly-rounded-divide-sqrt",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
]


def command(out: str = LIB) -> list[str]:
    return [HIPCC, *FLAGS, "-x", "hip", *SOURCES, "-o", out]


def build(force: bool = True, verbose: bool = False) -> str:
    """Compile the library (always, unless force=False and it is up to date)."""
    if not force and os.path.exists(LIB):
        newest = max(os.path.getmtime(p) for p in SOURCES + HEADERS)
        if os.path.getmtime(LIB) >= newest:
            return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
