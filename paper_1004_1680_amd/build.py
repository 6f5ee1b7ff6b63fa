"""Build the HIP library ``libmhd.so`` for gfx950 in-tree with hipcc.

Every source is compiled with ``-ffp-contract=off`` (each product and sum is
rounded as written, so the FP64 tier reproduces a plain evaluation of the
scheme) and with packed FP32 instructions disabled.
"""
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libmhd.so")
ARCH = os.environ.get("MHD_OFFLOAD_ARCH", "gfx950")


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def command(out=LIB, extra=()):
    return ["hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
            "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-variable", "-Wno-unused-function",
            "-I", os.path.join(ROOT, "include"), *extra, "-o", out, *sources()]


def build(verbose=True):
    cmd = command()
    if verbose:
        print(" ".join(cmd), flush=True)
    tmp = LIB + ".tmp"
    cmd[-len(sources()) - 1] = tmp
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
