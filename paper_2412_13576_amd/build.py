"""Builds the gfx950 shared library libgraver.so in-tree with hipcc.

Every HIP source is compiled for gfx950 only, with packed-FP32 instruction
selection disabled.  Sources whose arithmetic must be a plain binary64
evaluation (the reproducible descent, the start generator and the
augmentation) are compiled with -ffp-contract=off.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgraver.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["-O3", "-fPIC", "-std=c++17", "--offload-arch=gfx950",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", INCLUDE, "-I", CSRC, "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]
SOURCES = {
    "abi.cpp": ["-x", "hip"],
    "lattice.cpp": ["-x", "hip"],
    "pool.hip": [],
    "descent_fp64.hip": ["-ffp-contract=off"],
    "descent_f32.hip": ["-ffp-contract=fast"],
    "descent_big.hip": ["-ffp-contract=fast"],
    "descent_sparse.hip": ["-ffp-contract=fast"],
    "filter.hip": [],
    "augment.hip": ["-ffp-contract=off"],
    "extract.cpp": ["-x", "hip"],
    "solve.cpp": ["-x", "hip"],
    "inequality.cpp": ["-x", "hip"],
    "server.cpp": ["-x", "hip", "-pthread"],
}


def _compile(name: str) -> str:
    src = os.path.join(CSRC, name)
    obj = os.path.join(BUILD, name + ".o")
    cmd = [HIPCC, *COMMON, *SOURCES[name], "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, sorted(SOURCES)))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", "-o", tmp, *objs,
           "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
