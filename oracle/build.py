"""Build the FP64 CPU oracle (test infrastructure) into oracle/liboracle_btrt.so.

Plain gcc -O2, FP64, no fast-math, no FMA contraction, OpenMP over rows.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "btrt_oracle.c"), os.path.join(HERE, "btrt3_oracle.c")]
LIB = os.path.join(HERE, "liboracle_btrt.so")

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
          "-fno-fast-math", "-Wall", "-Wextra"]


def build(verbose: bool = False) -> str:
    """Compile the oracle; returns the path of the shared library."""
    cmd = ["gcc", *CFLAGS, *SRCS, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
