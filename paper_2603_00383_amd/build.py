"""Build step of the HIP library: compiles csrc/ into libseas.so for gfx950.

    python -m paper_2603_00383_amd.build        (or __graft_entry__.build())

Host build code (csrc/build.cpp) is plain C++ with OpenMP and strict IEEE
evaluation (-ffp-contract=off) so that integer decisions taken from floating
point (windows, admissibility) do not depend on contraction; the HIP sources are
compiled for gfx950 only, with packed FP32 instructions disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libseas.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
OMP_LIBDIR = os.path.join(ROCM, "lib", "llvm", "lib")

COMMON = ["-O3", "-fPIC", "-std=c++17", "-I" + INCLUDE, "-I" + CSRC, "-fopenmp"]
HIP_FLAGS = ["-x", "hip", "--offload-arch=gfx950", "-ffp-contract=fast",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
HOST_FLAGS = ["-x", "c++", "-ffp-contract=off", "-march=x86-64-v2"]

SOURCES = [("build.cpp", HOST_FLAGS), ("kernels.hip", HIP_FLAGS), ("kernels_x16.hip", HIP_FLAGS),
           ("api.hip", HIP_FLAGS), ("server.hip", HIP_FLAGS)]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("compile failed: " + " ".join(cmd[:8]) + " ...")
    return r


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src, flags in SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        _run([HIPCC] + COMMON + flags + ["-c", os.path.join(CSRC, src), "-o", obj], verbose)
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fopenmp", "--offload-arch=gfx950", "-o", tmp] + objs +
         ["-L" + OMP_LIBDIR, "-Wl,-rpath," + OMP_LIBDIR], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
