"""Build the native libraries in-tree.

  libmggen.so  host problem generator (g++ -O3 -fopenmp)
  libmgq1.so   HIP solver library for gfx950 (hipcc --offload-arch=gfx950)

Run as `python -m paper_2405_05047_amd.build` (or call build_all()).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB_GEN = os.path.join(HERE, "libmggen.so")
LIB_MG = os.path.join(HERE, "libmgq1.so")

HIP_SOURCES = ["mgq1_kernels.hip", "mgq1_runtime.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _run(cmd):
    print("+", " ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build_gen():
    src = os.path.join(CSRC, "gen", "mggen.cpp")
    _run(["g++", "-O3", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
          "-Wall", "-Wextra", "-I", INCLUDE, src, "-o", LIB_GEN + ".tmp"])
    os.replace(LIB_GEN + ".tmp", LIB_GEN)


def build_hip():
    srcs = [os.path.join(CSRC, s) for s in HIP_SOURCES]
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-ffp-contract=on", "-Wall",
           "-I", INCLUDE] + srcs + ["-o", LIB_MG + ".tmp"]
    _run(cmd)
    os.replace(LIB_MG + ".tmp", LIB_MG)


def build_all():
    build_gen()
    build_hip()


if __name__ == "__main__":
    what = sys.argv[1:] or ["all"]
    if "gen" in what:
        build_gen()
    if "hip" in what:
        build_hip()
    if "all" in what:
        build_all()
