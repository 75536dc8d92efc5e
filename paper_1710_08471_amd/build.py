"""Build libcqr2.so (HIP, gfx950 only) in-tree with hipcc.

Usage: python -m paper_1710_08471_amd.build   (or build() from Python).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libcqr2.so")
SOURCES = ["cqr2_gram.hip", "cqr2_cholinv.hip", "cqr2_apply.hip", "cqr2_gemm.hip", "cqr2_wide.hip", "cqr2_driver.hip",
           "cqr2_step.hip", "cqr2_serve.hip", "cqr2_api.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (need ROCm)")


def build(verbose: bool = False) -> str:
    """Compile every HIP source into one shared library; returns its path."""
    out_tmp = LIB + ".tmp"
    cmd = [
        hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
        # packed FP32 instructions are kept out of all generated code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        f"-I{INCLUDE}",
        *[os.path.join(CSRC, s) for s in SOURCES],
        "-o", out_tmp,
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed with status {res.returncode}")
    os.replace(out_tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
