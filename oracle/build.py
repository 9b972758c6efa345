"""Compile the CPU oracle (plain C) into oracle/libmdref.so.

TEST INFRASTRUCTURE ONLY: the oracle checks the GPU path and is never used by it.
-ffp-contract=off keeps every multiply and add a separately rounded operation,
so the pair predicate is exactly the sequence of roundings written in mdref.c.
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mdref.c")
LIB = os.path.join(HERE, "libmdref.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
