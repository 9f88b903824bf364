"""Compile the C oracle (test infrastructure) into oracle/librsi_oracle.so.

Flags: binary64 arithmetic exactly as written -- no contraction into fused
multiply-add (-ffp-contract=off), no fast-math -- and OpenMP over rays.  No
-march flag: the library must run on whichever x86-64 host loads it.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rsi_oracle.c")
LIB = os.path.join(HERE, "librsi_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-std=c11", "-O3", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
           SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
