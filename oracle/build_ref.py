"""Build the C half of the oracle (oracle/ebc_ref.c -> oracle/libebc_ref.so).

Test infrastructure: the oracle is a checker, not part of the product path.
Plain gcc with OpenMP; x86-64-v3 so that the shared object also runs on the
benchmark host's CPU.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ebc_ref.c")
LIB = os.path.join(HERE, "libebc_ref.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-std=c99", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared",
           SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
