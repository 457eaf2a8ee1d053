"""Build the HIP library libdvm.so for gfx950 (in-tree).

hipcc compiles every source for gfx950 only.  Packed FP32 instructions are
disabled (-packed-fp32-ops): the kernels are written as scalar FP32/FP64 code.
Run: python -m paper_1503_00707_amd.build
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libdvm.so")
SOURCES = ["csrc/mesh.cpp", "csrc/solver.cpp", "csrc/batch.cpp", "csrc/sensor.cpp", "csrc/persist.cpp", "csrc/korobov.cpp", "csrc/lbm.cpp", "csrc/kernels_misc.hip",
           "csrc/kernels_f32.hip", "csrc/kernels_f64.hip", "csrc/sensor.hip", "csrc/korobov.hip", "csrc/lbm.hip", "csrc/adapt.hip"]


def build(verbose: bool = False, jobs: int = 3) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    flags = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(bdir, os.path.basename(src) + ".o")
        objs.append(obj)
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [hipcc, *flags, *lang, "-c", os.path.join(HERE, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        if len(procs) >= jobs:
            if procs.pop(0).wait():
                raise RuntimeError("hipcc failed")
    for p in procs:
        if p.wait():
            raise RuntimeError("hipcc failed")
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
