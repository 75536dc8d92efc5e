"""Build libcqr2.so (HIP, gfx950 only) in-tree with hipcc.

Each source is compiled to an object on its own (in parallel), then the
objects are linked into one shared library.

Usage: python -m paper_1710_08471_amd.build   (or build() from Python).
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libcqr2.so")
OBJDIR = os.path.join(ROOT, "_build")
SOURCES = ["cqr2_gram.hip", "cqr2_cholinv.hip", "cqr2_apply.hip", "cqr2_gemm.hip", "cqr2_wide.hip", "cqr2_stream16.hip", "cqr2_driver.hip",
           "cqr2_step.hip", "cqr2_serve.hip", "cqr2_api.hip"]
ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are kept out of all generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (need ROCm)")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed with status {res.returncode}: {' '.join(cmd[-3:])}")


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every HIP source and link them into one shared library; returns its path."""
    os.makedirs(OBJDIR, exist_ok=True)
    cc = hipcc()
    objs = []
    cmds = []
    for s in SOURCES:
        obj = os.path.join(OBJDIR, os.path.splitext(s)[0] + ".o")
        objs.append(obj)
        cmds.append([cc, *FLAGS, f"-I{INCLUDE}", "-c", os.path.join(CSRC, s), "-o", obj])
    jobs = jobs or min(len(cmds), max(1, min(16, os.cpu_count() or 1)))
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        for f in [ex.submit(_run, c, verbose) for c in cmds]:
            f.result()
    out_tmp = LIB + ".tmp"
    _run([cc, *FLAGS, "-shared", *objs, "-o", out_tmp], verbose)
    os.replace(out_tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
