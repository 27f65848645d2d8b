"""Compile the FP64 CPU oracle (test infrastructure) into oracle/libftc_oracle.so.

gcc, C11, OpenMP, no fast-math, and -ffp-contract=off so that every product
and sum is rounded as written.  No -march=native: the library is built here
and also loaded on other hosts."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ftc_oracle.c")
LIB = os.path.join(HERE, "libftc_oracle.so")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
