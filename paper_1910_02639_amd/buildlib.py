"""Compiles libbtree.so (the HIP kernels and the C ABI) for gfx950, in-tree."""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libbtree.so")
SOURCES = ["scan.hip", "sort.hip", "build.hip", "find.hip", "api.hip", "batch.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # The FP64 predicate and Eq. 2 must be evaluated with every operation
    # rounded: no contraction into fused multiply-adds.
    "-ffp-contract=off",
    # Packed FP32 VALU instructions stay disabled.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # roctx ranges around the phases of the entry points.
    "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx",
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc, *HIPCC_FLAGS, "-I" + INCLUDE, *[os.path.join(CSRC, s) for s in SOURCES],
           "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stdout + r.stderr)
    if verbose:
        print(r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=False))
