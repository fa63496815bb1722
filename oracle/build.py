"""Build the FP64 oracle (test infrastructure) into oracle/liborc.so with gcc.

IEEE double throughout: no -ffast-math, no FMA contraction.  OpenMP runs the
independent loops over particles on orc_set_threads() threads (default 1), with
results bit-identical to one thread.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liborc.so")


def build(verbose: bool = False) -> str:
    cmd = [
        "gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
        "-Wall", "-Wextra", "-o", LIB, os.path.join(HERE, "orc.c"), "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
