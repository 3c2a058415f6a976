"""Build the HIP library (libtreeray.so) in-tree for gfx950 with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtreeray.so")
SOURCES = ["runtime.hip", "tree.hip", "rays.hip", "trace.hip", "dust.hip", "mlp.hip", "fixed_point.hip", "uv.hip"]
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off",                      # fixed FP64 operation order in the tree build
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-mllvm", "-amdgpu-mfma-vgpr-form",       # matrix-core results in VGPRs: no accumulator reads
                                              # before the activations (guess network)
    "-Wno-unused-result", "-Wno-unused-value",
    "-I", os.path.join(ROOT, "include"), "-I", SRC,
]


def hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.exists(c) or c == "hipcc":
            return c
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(SRC, s) for s in SOURCES]
    cmd = [hipcc()] + FLAGS + srcs + ["-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
