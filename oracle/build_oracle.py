"""Build the FP64 CPU oracle (test infrastructure) into oracle/libbm_oracle.so.

Plain gcc, -O2, no fast-math and no FP contraction, so every operation is the
IEEE double operation written in bm_oracle.c.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libbm_oracle.so")


def build(verbose=False):
    src = os.path.join(HERE, "bm_oracle.c")
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
           "-Wall", "-Wextra", "-fPIC", "-shared", "-o", LIB, src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
