"""Builds libhsvd.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_1008_1371_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libhsvd.so")
BUILD_DIR = os.path.join(ROOT, "_build")

SOURCES = ["api.hip", "pair_kernels.hip", "block_kernels.hip", "mixed_kernels.hip", "batch_kernels.hip",
           "gemm_kernels.hip", "batch_persist.hip", "wide_kernels.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # every FMA in the library is written out; no contraction elsewhere
    "-ffp-contract=off",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # MFMA accumulators in ordinary VGPRs: keeps loop-carried accumulators
    # from being copied between register files on every iteration
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-I" + os.path.join(ROOT, "include"),
    "-Wall", "-Wno-unused-result",
]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


GEN_SRC = os.path.join(CSRC, "gen_indefinite.c")
GEN_LIB = os.path.join(HERE, "libhsvd_gen.so")


def build_gen() -> str:
    """Host library of the extended-precision test-matrix generator (gcc,
    OpenMP; x87 long double)."""
    tmp = GEN_LIB + ".tmp"
    cmd = [os.environ.get("CC", "gcc"), "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", GEN_SRC, "-o", tmp, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"gcc failed for gen_indefinite.c:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, GEN_LIB)
    return GEN_LIB


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    build_gen()
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "--offload-arch=gfx950", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
