"""Builds libmc.so in-tree for gfx950.

The host network builder is plain C++/OpenMP (g++); the kernels and the C
interface are HIP (hipcc --offload-arch=gfx950).  Both are compiled without
floating-point contraction so that every rounding step is the one the
specification writes down.  Packed FP32 instructions are disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libmc.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall", "-Wno-unused-result"]
CXX_FLAGS = ["-O3", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-Wall"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(line for line in r.stdout.splitlines() if "packed-fp32-ops" not in line)
    if r.returncode != 0:
        sys.stderr.write(out + "\n")
        raise RuntimeError("build step failed: " + " ".join(cmd))
    return out


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    inc = ["-I" + INCLUDE, "-I" + CSRC]
    objs = []
    o = os.path.join(BUILD, "mc_build.o")
    _run(["g++", *CXX_FLAGS, *inc, "-c", os.path.join(CSRC, "mc_build.cpp"), "-o", o])
    objs.append(o)
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    for src in ("mc_kernels.hip", "mc_persist.hip", "mc_replay.hip", "mc_adjoint.hip", "mc_owner.hip", "mc_bucket.hip", "mc_construct.hip",
                "mc_noalloc.hip", "mc_api.hip"):
        o = os.path.join(BUILD, src.replace(".hip", ".o"))
        out = _run([hipcc, *HIP_FLAGS, *inc, "-c", os.path.join(CSRC, src), "-o", o])
        if verbose and out.strip():
            print(out)
        objs.append(o)
    tmp = LIB + ".tmp"
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs, "-lgomp"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
