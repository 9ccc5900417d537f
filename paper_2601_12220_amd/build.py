"""Build libbes.so in-tree: host C++ with g++, HIP sources with hipcc for gfx950.

Usage: python -m paper_2601_12220_amd.build   (always recompiles everything)
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libbes.so")
ARCH = os.environ.get("BES_OFFLOAD_ARCH", "gfx950")

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
CXX = shutil.which("g++") or "g++"

HIP_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions stay disabled on this target
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-Wextra", "-Wno-unused-parameter"]


def _run(cmd):
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if res.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + res.stdout)
    return res.stdout


def sources():
    host = sorted(glob.glob(os.path.join(CSRC, "host", "*.cpp")))
    hip_host = [os.path.join(CSRC, "abi.cpp")]
    kernels = sorted(glob.glob(os.path.join(CSRC, "kernels", "*.hip")))
    return host, hip_host, kernels


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    host, hip_host, kernels = sources()
    jobs = []
    for src in host:
        obj = os.path.join(OBJ, os.path.basename(src) + ".o")
        jobs.append([CXX, *HOST_FLAGS, "-c", src, "-o", obj])
    for src in hip_host:
        obj = os.path.join(OBJ, os.path.basename(src) + ".o")
        jobs.append([HIPCC, "-O2", "-std=c++17", "-fPIC", "-Wall", "-x", "hip",
                     f"--offload-arch={ARCH}", "-c", src, "-o", obj])
    for src in kernels:
        obj = os.path.join(OBJ, os.path.basename(src) + ".o")
        jobs.append([HIPCC, *HIP_FLAGS, "-x", "hip", "-c", src, "-o", obj])
    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        outs = list(ex.map(_run, jobs))
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    objs = [j[-1] for j in jobs]
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
