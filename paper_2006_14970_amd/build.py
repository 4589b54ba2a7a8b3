"""Build libfge.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2006_14970_amd.build

Every source is compiled for gfx950 only, with packed-FP32 instruction selection disabled, and
linked into ``paper_2006_14970_amd/libfge.so`` next to this file.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libfge.so")
BUILD_DIR = os.path.join(ROOT, "_build")

SOURCES = ["fge_plan.cpp", "fge_api.cpp", "fge_batch.cpp", "fge_server.cpp", "fge_tune.cpp", "fge_kernels.hip", "fge_util.hip", "fge_converge.hip", "fge_closed_form.hip"]
ARCH = "gfx950"
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP toolchain is required to build libfge")


def _compile(cc: str, src: str, verbose: bool) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD_DIR, src + ".o")
    cmd = [cc, "-x", "hip", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
           "-Wall", "-Wno-unused-function", *DEVICE_FLAGS, "-I", INCLUDE, "-I", CSRC,
           "-c", path, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return obj


def build(verbose: bool = False) -> str:
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(BUILD_DIR, exist_ok=True)
    cc = hipcc()
    # The sources compile independently; the kernel file dominates, so start it first.
    order = sorted(SOURCES, key=lambda f: os.path.getsize(os.path.join(CSRC, f)), reverse=True)
    jobs = max(1, min(len(order), os.cpu_count() or 1, 8))
    with ThreadPoolExecutor(jobs) as pool:
        done = dict(zip(order, pool.map(lambda f: _compile(cc, f, verbose), order)))
    objs = [done[f] for f in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("linking libfge.so failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
