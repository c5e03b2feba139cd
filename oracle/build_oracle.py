"""Build the oracle's shared library (test infrastructure only).

Compiles ``lrbg_oracle.c`` with gcc and OpenMP, without floating-point
contraction or fast-math, so that each product is rounded before it is
added.  The result is ``liblrbg_oracle.so`` next to this file.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lrbg_oracle.c")
LIB = os.path.join(HERE, "liblrbg_oracle.so")

CFLAGS = ["-O2", "-fPIC", "-shared", "-std=c99", "-fopenmp",
          "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra"]


def build(verbose: bool = False) -> str:
    cmd = ["gcc", *CFLAGS, SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
