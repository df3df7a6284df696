"""Builds libheston.so for gfx950 with hipcc, in-tree.

Usage: python -m paper_2309_10477_amd.build   (or call build()).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = [os.path.join(HERE, "csrc", f) for f in ("api.hip", "price_kernel.hip",
                                               "adjoint_kernel.hip", "batch_kernel.hip",
                                               "batch_api.hip", "server.hip")]
HDRS = [os.path.join(HERE, "csrc", f) for f in ("internal.hpp", "device_math.hpp",
                                                "path_step.hpp")] + \
    [os.path.join(os.path.dirname(HERE), "include", "heston.h")]
LIB = os.path.join(HERE, "libheston.so")
ARCH = os.environ.get("HESTON_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc, *FLAGS, "-o", tmp, *SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
