"""Build the HIP library ``libmhd.so`` for gfx950 in-tree with hipcc.

Every source is built with ``-ffp-contract=off``: the compiler forms no
fused multiply-add by itself, so the FP64 tier rounds every product and sum
as written, and the FP32 tier uses exactly the fused multiply-adds its
shared device functions spell out (the same in every kernel, which keeps
the x, y and z sweeps bitwise symmetric).  Packed FP32 instructions are
disabled for every source.
"""
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libmhd.so")
BUILD = os.path.join(ROOT, "_build")
ARCH = os.environ.get("MHD_OFFLOAD_ARCH", "gfx950")


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def compile_command(src, obj):
    return ["hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-c",
            "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang",
            "-packed-fp32-ops", "-Wall", "-Wno-unused-variable", "-Wno-unused-function",
            "-I", os.path.join(ROOT, "include"), "-o", obj, src]


def build(verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    procs = []
    for src in sources():
        obj = os.path.join(BUILD, os.path.basename(src).replace(".hip", ".o"))
        cmd = compile_command(src, obj)
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        objs.append(obj)
    for p in procs:
        if p.wait() != 0:
            raise RuntimeError("hipcc failed")
    tmp = LIB + ".tmp"
    link = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
