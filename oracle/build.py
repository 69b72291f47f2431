"""Build the FP64 CPU oracle (test infrastructure only) into oracle/_liboracle.so.

The flags target x86-64-v3 (AVX2/FMA) so that the library built here also loads on
the host CPU of the machine that runs the GPU tests.  No intrinsics are used; the
compiler vectorises what it can.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "_liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = [
        "gcc", "-std=gnu11", "-O2", "-march=x86-64-v3", "-fopenmp", "-fcx-limited-range",
        "-fPIC", "-shared", "-o", LIB + ".tmp", SRC, "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
