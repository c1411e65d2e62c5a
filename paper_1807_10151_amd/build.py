"""Builds libsuppcg.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1807_10151_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsuppcg.so")

SOURCES = ["projector.hip", "fft.hip", "tv.hip", "cg.hip", "learned.hip", "noalloc.hip", "quality.hip", "stored.hip", "art.hip",
           "geometry.cpp", "capi.cpp"]

# -ffp-contract=off: no multiply and add is fused implicitly; the fused ones
# are the explicit fma calls, so a formula evaluated on the host and on the
# device (the bin positions of the axis-parallel weights) rounds the same way.
# -packed-fp32-ops: no packed FP32 instructions are generated.
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *FLAGS, "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libsuppcg.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
