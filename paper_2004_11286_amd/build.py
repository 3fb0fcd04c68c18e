"""Build libmclbm.so for gfx950 in-tree (hipcc cross-compiles without a GPU).

Usage: python -m paper_2004_11286_amd.build [-v]
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libmclbm.so")
BUILD_DIR = os.path.join(HERE, "_build")

SOURCES = ["mclbm.hip", "nn.hip", "inst_fp64.hip", "inst_fp32_fp64.hip", "inst_weak.hip", "inst_cvt.hip",
           "inst_weak_cvt.hip", "inst_fp32.hip", "inst_fp16.hip", "inst_bf16.hip", "inst_i16.hip", "inst_jets.hip"]

ARCH = os.environ.get("MCLBM_OFFLOAD_ARCH", "gfx950")
# Packed FP32 instructions are switched off for all device code.
HIPFLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-Wno-unused-command-line-argument"]


def hipcc() -> str:
    for cand in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libmclbm)")


def _compile(src: str, verbose: bool, extra: list[str]) -> str:
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *HIPFLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    if verbose and (r.stderr.strip()):
        print(r.stderr)
    if extra:
        with open(obj + ".remarks", "w") as fh:      # compiler remarks (register usage)
            fh.write(r.stderr)
    return obj


def build_library(verbose: bool = False, resource_usage: bool = False, jobs: int | None = None) -> str:
    """Compile every translation unit in parallel and link libmclbm.so."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    extra = ["-Rpass-analysis=kernel-resource-usage"] if resource_usage else []
    jobs = jobs or min(len(SOURCES), max(1, (os.cpu_count() or 2)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, extra), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose="-v" in sys.argv, resource_usage="-r" in sys.argv))
