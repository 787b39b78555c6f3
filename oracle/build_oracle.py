"""Build the FP64 CPU oracle (test infrastructure).

Two libraries from the same source, both plain gcc -O2 with no fast-math and
no FP contraction, so every operation is the IEEE double operation written in
bm_oracle.c:
  oracle/libbm_oracle.so      single-threaded (correctness runs);
  oracle/libbm_oracle_omp.so  OpenMP over independent per-point loops, every
                              sum still taken in index order by one thread, so
                              its results are bit-identical (timing on all host
                              cores, stored results of large workloads).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libbm_oracle.so")
LIB_OMP = os.path.join(HERE, "libbm_oracle_omp.so")
SRC = os.path.join(HERE, "bm_oracle.c")
FLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra", "-fPIC",
         "-shared"]


def build(verbose=False):
    for out, extra in ((LIB, ["-Wno-unknown-pragmas"]), (LIB_OMP, ["-fopenmp"])):
        cmd = ["gcc", *FLAGS, *extra, "-o", out + ".tmp", SRC, "-lm"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
