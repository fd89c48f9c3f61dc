"""Build step for the CPU oracle (test infrastructure).

Compiles oracle.c with gcc into liboracle.so next to this file:
-O2, no FP contraction, SSE2 arithmetic, no fast-math, OpenMP for the one
element-parallel variant.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
          "-fno-fast-math", "-msse2", "-mfpmath=sse", "-fopenmp",
          "-Wall", "-Wextra", "-Werror"]


def build(out=LIB, src=None, verbose=False):
    """Compile the oracle (or, for the tests that plant mistakes in a copy of
    it, the source file `src`) into the shared library `out`."""
    src = src or os.path.join(HERE, "oracle.c")
    cmd = ["gcc", *CFLAGS, "-I", HERE, src, "-o", out + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
