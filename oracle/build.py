"""Build the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so.

Plain gcc, no FMA contraction (the default x86-64 target has none), OpenMP
over cells.  Run: python oracle/build.py
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "dvm_oracle.c")
    cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wno-unused-function", src, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
