"""Build the native libraries in-tree.

  libmggen.so  host problem generators (g++ -O3 -fopenmp): adaptive Q1 hierarchies and the
               explicit pressure-correction workload
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

HIP_SOURCES = ["mgq1_kernels.hip", "mgq1_batch.hip", "mgq1_runtime.hip", "mgq1_time.hip", "mgq1_cheb.hip",
               "mgq1_ns.hip", "mgq1_asm.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _run(cmd):
    print("+", " ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build_gen():
    srcs = [os.path.join(CSRC, "gen", "mggen.cpp"), os.path.join(CSRC, "gen", "mgns.cpp")]
    _run(["g++", "-O3", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
          "-Wall", "-Wextra", "-I", INCLUDE] + srcs + ["-o", LIB_GEN + ".tmp"])
    os.replace(LIB_GEN + ".tmp", LIB_GEN)


def build_hip():
    """Compile the HIP translation units in parallel (the kernel units dominate), then link."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    flags = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-ffp-contract=on", "-Wall", "-I", INCLUDE]
    procs, objs = [], []
    for src in HIP_SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC] + flags + ["-c", os.path.join(CSRC, src), "-o", obj]
        print("+", " ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        objs.append(obj)
    failed = [p.args for p in procs if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", LIB_MG + ".tmp"])
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
