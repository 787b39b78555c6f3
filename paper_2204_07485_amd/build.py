"""Build libbigmeans.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2204_07485_amd.build [-v]

Packed FP32 instructions are disabled for the device code (the library's
kernels are written for scalar FP32/FP64 VALU and never rely on them).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbigmeans.so")
SOURCES = ["bm_api.hip", "bm_solver.hip", "bm_assign.hip", "bm_assign_mfma.hip", "bm_assign_mfma32.hip",
           "bm_batch.hip", "bm_serve.hip",
           "bm_noalloc.hip"]
ARCH = os.environ.get("BM_OFFLOAD_ARCH", "gfx950")


def hipcc_flags():
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I" + os.path.join(ROOT, "include")]


def build(verbose=False, jobs=4):
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        objs.append(obj)
        cmd = ["hipcc", *hipcc_flags(), "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd)))
        if len(procs) >= jobs:
            name, p = procs.pop(0)
            if p.wait() != 0:
                raise RuntimeError(f"hipcc failed on {name}")
    for name, p in procs:
        if p.wait() != 0:
            raise RuntimeError(f"hipcc failed on {name}")
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
