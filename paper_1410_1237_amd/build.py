"""Builds the native parts in-tree:

* ``liblouvain.so``  -- the HIP library for gfx950 (csrc/*.hip), C ABI in include/louvain.h
* ``_graphgen.so``   -- the seeded input generator (plain C, OpenMP)

Run ``python -m paper_1410_1237_amd.build`` or call ``build_all()``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "liblouvain.so")
GEN_LIB = os.path.join(PKG, "_graphgen.so")
SOURCES = ["prims.hip", "graph.hip", "sweep.hip", "color.hip", "batch.hip", "api.hip", "serve.hip"]
ARCH = os.environ.get("LOUVAIN_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
    # packed-FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r


def build_hip(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = []

    def one(src):
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        _run([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 4)) as ex:
        objs = list(ex.map(one, SOURCES))
    tmp = LIB + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def build_gen(verbose: bool = False) -> str:
    tmp = GEN_LIB + ".tmp"
    _run(["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", "-o", tmp, os.path.join(PKG, "graphgen.c"), "-lm"])
    os.replace(tmp, GEN_LIB)
    if verbose:
        print("built", GEN_LIB)
    return GEN_LIB


def build_all(verbose: bool = False):
    build_gen(verbose)
    build_hip(verbose)


if __name__ == "__main__":
    build_all(verbose=True)
    sys.exit(0)
