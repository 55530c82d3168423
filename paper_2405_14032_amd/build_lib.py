"""Builds libopf.so (HIP for gfx950) in place, next to this file."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["csrc/opf_capi.hip", "csrc/opf_kernels.hip", "csrc/opf_symbolic.cpp", "csrc/opf_chol.hip",
           "csrc/opf_chol_symbolic.cpp", "csrc/opf_ipm.hip"]
LIB = os.path.join(HERE, "libopf.so")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    return "hipcc"


def build(verbose: bool = False) -> str:
    cmd = [
        hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
        # no packed-FP32 instructions anywhere in the device code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        # contraction decided per source expression, so every kernel that
        # shares an expression rounds it identically
        "-ffp-contract=on",
        "-Wall", "-Wno-unused-result",
        "-o", LIB + ".tmp",
    ] + [os.path.join(HERE, s) for s in SOURCES] + [
        # the dense trailing updates of the pg chain's fronts in the sparse Cholesky
        "-L/opt/rocm/lib", "-lrocblas",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, cwd=HERE, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libopf.so")
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
