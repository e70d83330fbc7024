"""Build the CPU oracle shared library (plain gcc, OpenMP, no HIP).

The oracle is test infrastructure: only tests, the smoke check and the benchmark's CPU-baseline
leg load it.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    # -fcx-limited-range: textbook complex multiply/divide (no inf/nan recovery), values here are
    # always finite and far from overflow.
    cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fcx-limited-range", "-fPIC", "-shared",
           SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
