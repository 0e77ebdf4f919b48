"""Build the CPU oracle shared library (test infrastructure only).

The oracle is plain C compiled by gcc; it never links the GPU library.
Usage: python oracle/build.py   (or import and call build()).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

# Generic x86-64 code: the library is built in one place and run on another
# host, so no -march=native.  -ffp-contract=off keeps a*b+c as two roundings.
CFLAGS = ["-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared", "-Wall", "-Wextra"]


def build(verbose=False):
    cmd = ["gcc"] + CFLAGS + [SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
