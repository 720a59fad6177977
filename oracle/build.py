"""Compile the FP64 oracle (plain C, gcc) into oracle/liboracle.so.

Test infrastructure only: the product library never links or loads it.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "vesis_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

# Plain IEEE arithmetic: no fast-math and no FMA contraction, so every line
# of the oracle rounds exactly as written.
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
          "-fno-fast-math", "-Wall", "-Wno-unknown-pragmas"]


def build(verbose: bool = False, src: str = SRC, lib: str = LIB) -> str:
    tmp = lib + ".tmp"
    cmd = ["gcc", *CFLAGS, "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
