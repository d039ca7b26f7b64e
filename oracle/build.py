"""Build the FP64 CPU oracle (test infrastructure only) with gcc.

``-ffp-contract=off`` keeps the contact test d^2 < (r_i + r_j)^2 and the cell
hash free of fused multiply-adds, so they are evaluated exactly as written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dem_oracle.c")
LIB = os.path.join(HERE, "libdem_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O3", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-Wno-unused-parameter", SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
