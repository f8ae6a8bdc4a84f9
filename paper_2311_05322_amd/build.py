"""Builds libmx.so (the gfx950 solver library) in-tree.

HIP sources are compiled by hipcc for gfx950 with packed-FP32 instructions
disabled; the host C++ (topology, decomposition) by g++ with OpenMP.
Usage: python -m paper_2311_05322_amd.build [--jobs N]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmx.so")
ARCH = os.environ.get("MX_OFFLOAD_ARCH", "gfx950")

HIP_SOURCES = ["k_operator.hip", "k_dense.hip", "k_krylov.hip", "k_learned.hip", "k_block.hip", "mx_api.hip"]
CPP_SOURCES = ["host_mesh.cpp", "tune_cache.cpp", "block_lsq.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-result", "-I", os.path.join(ROOT, "include"), "-I", CSRC]
CXX_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-fopenmp", "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _run(cmd):
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + p.stdout + p.stderr)
    return p


def build(jobs: int | None = None, verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    cmds = []
    objs = []
    for src in HIP_SOURCES:
        o = os.path.join(OBJ, src + ".o")
        objs.append(o)
        cmds.append([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", o])
    for src in CPP_SOURCES:
        o = os.path.join(OBJ, src + ".o")
        objs.append(o)
        cmds.append(["g++", *CXX_FLAGS, "-c", os.path.join(CSRC, src), "-o", o])
    with cf.ThreadPoolExecutor(max_workers=jobs or min(8, os.cpu_count() or 4)) as ex:
        for p in ex.map(_run, cmds):
            if verbose and (p.stdout or p.stderr):
                print(p.stdout + p.stderr)
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs, "-lgomp"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("-v", action="store_true")
    a = ap.parse_args()
    print(build(a.jobs, a.v))
    sys.exit(0)
