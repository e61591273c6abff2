"""Build the HIP library ``libhlb.so`` in-tree for gfx950.

hipcc compiles every source of ``csrc/`` into one shared library exposing the
C-ABI of ``include/hlb.h``.  Packed-FP32 instructions are disabled for all
device code.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhlb.so")

SOURCES = ["kernels.hip", "batch.hip", "nn.hip", "hlb_api.cpp", "batch_api.cpp", "nn_api.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]


def build(verbose: bool = False) -> str:
    srcs = []
    for s in SOURCES:
        p = os.path.join(CSRC, s)
        # hipcc treats .cpp as host C++ unless told it is HIP
        srcs += (["-x", "hip", p] if s.endswith(".hip") else ["-x", "hip", p])
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
