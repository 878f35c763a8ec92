"""Build libz4c.so (HIP, gfx950) in-tree with hipcc.

The library is compiled for gfx950 only.  Packed-FP32 instruction selection
is disabled (-packed-fp32-ops): some forms have produced silently wrong
results on these parts.  FP64 arithmetic uses hipcc's default contraction;
the pi-mirror symmetry of the results does not depend on it because every
mirror pair runs the same instruction stream.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libz4c.so")
SOURCES = [os.path.join(CSRC, "z4c_kernels.hip"), os.path.join(CSRC, "z4c_constraints.hip"),
           os.path.join(CSRC, "z4c_hierarchy.hip"), os.path.join(CSRC, "z4c_api.hip")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", INCLUDE, "-I", CSRC]


def build(verbose: bool = False) -> str:
    """Compile every source into paper_2607_08743_amd/libz4c.so (always recompiles)."""
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, os.path.basename(src) + ".o")
        cmd = [HIPCC] + FLAGS + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        objs.append(obj)
    for p in procs:
        if p.wait() != 0:
            raise RuntimeError("hipcc failed building libz4c.so")
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
