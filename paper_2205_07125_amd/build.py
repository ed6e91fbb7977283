"""Builds libsnn.so for gfx950: the HIP kernels and runtime (hipcc) plus the
host setup and the seeded generator (gcc/g++ with OpenMP).  Always compiles
from source; the library lands next to this file."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INC = os.path.join(ROOT, "include")
SYNTH = os.path.join(ROOT, "synth")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libsnn.so")

ARCH = os.environ.get("SNN_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# -ffp-contract=off: the membrane update rounds after every operation.
# -packed-fp32-ops off: no packed FP32 instructions are emitted.
HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-ffp-contract=off",
    "-fno-gpu-flush-denormals-to-zero", "-munsafe-fp-atomics",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument", "-I", INC, "-I", CSRC,
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    o = os.path.join(BUILD, "synth.o")
    _run(["gcc", "-O2", "-fopenmp", "-fPIC", "-std=c11", "-c", os.path.join(SYNTH, "synth.c"),
          "-o", o], verbose)
    objs.append(o)
    o = os.path.join(BUILD, "snn_setup.o")
    _run(["g++", "-O2", "-fopenmp", "-fPIC", "-std=c++17", "-Wall", "-I", INC, "-I", SYNTH, "-c",
          os.path.join(CSRC, "snn_setup.cpp"), "-o", o], verbose)
    objs.append(o)
    for src in ("snn_kernels.hip", "snn_runtime.hip"):
        o = os.path.join(BUILD, src.replace(".hip", ".o"))
        _run([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", o], verbose)
        objs.append(o)
    tmp = LIB + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lgomp"],
         verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
