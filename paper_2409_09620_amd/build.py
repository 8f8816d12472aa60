"""Builds the HIP library in-tree: paper_2409_09620_amd/_lib/liboedg.so (gfx950)."""

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIBDIR = os.path.join(HERE, "_lib")
LIB = os.path.join(LIBDIR, "liboedg.so")

ARCH = os.environ.get("OEDG_OFFLOAD_ARCH", "gfx950")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
# packed FP32 instructions are disabled for every HIP translation unit
HIP_FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", INCLUDE, "-I", CSRC]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    objs = []
    # host-side mesh precompute: no FMA contraction, so lengths and sorts are reproducible
    o = os.path.join(BUILD, "mesh_host.o")
    _run(["g++", "-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-I", CSRC, "-I", INCLUDE,
          "-c", os.path.join(CSRC, "mesh_host.cpp"), "-o", o], verbose)
    objs.append(o)
    o = os.path.join(BUILD, "schedule.o")
    _run(["g++", "-O2", "-std=c++17", "-fPIC", "-I", CSRC, "-I", INCLUDE,
          "-c", os.path.join(CSRC, "schedule.cpp"), "-o", o], verbose)
    objs.append(o)
    for src in ("kernels.hip", "capi.hip", "batch.hip"):
        o = os.path.join(BUILD, src.replace(".hip", ".o"))
        _run([HIPCC] + HIP_FLAGS + ["-c", os.path.join(CSRC, src), "-o", o], verbose)
        objs.append(o)
    tmp = LIB + f".tmp{os.getpid()}"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs, verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
