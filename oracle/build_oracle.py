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


def build_sanitized(out: str, verbose: bool = False) -> str:
    """The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
    (ROCm's clang, whose shared sanitizer runtime the GPU library's sanitized
    host build uses too, so both load into one process), for CPU tests."""
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cc = os.path.join(rocm, "llvm", "bin", "clang")
    cmd = [cc, "-O1", "-g", "-fPIC", "-shared", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-shared-libasan", SRC, "-o", out,
           "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
