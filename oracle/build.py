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


def build_timing(out_dir, openmp=False, verbose=False):
    """A timing build of the same source for the CPU baseline, compiled on the
    host that runs it: -O3 -march=native (still -ffp-contract=off), and with
    openmp the annotated loops over all cores.  Returns the library path."""
    name = "liboracle_native_omp.so" if openmp else "liboracle_native.so"
    out = os.path.join(out_dir, name)
    flags = ["-O3", "-march=native", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared"]
    if openmp:
        flags.append("-fopenmp")
    cmd = ["gcc"] + flags + [SRC, "-o", out + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


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
