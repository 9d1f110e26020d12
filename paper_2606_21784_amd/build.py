"""Compile the HIP library libcae.so for gfx950 (in-tree, next to this file)."""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = [os.path.join(HERE, "csrc", "cae_engine.hip")]
EXTRA = [os.path.join(HERE, "csrc", "cae_mlp.hip")]
LIB = os.path.join(HERE, "libcae.so")
UBENCH_SRC = os.path.join(HERE, "csrc", "cae_ubench.hip")
UBENCH_LIB = os.path.join(HERE, "libcae_ubench.so")
ARCH = "gfx950"


def hipcc():
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def command(out, srcs=None):
    if srcs is None:
        srcs = SOURCES + [s for s in EXTRA if os.path.exists(s)]
    return [hipcc(), "-O3", "-std=c++17", "--offload-arch=" + ARCH, "-fPIC", "-shared",
            "-ffp-contract=off",
            # packed fp32 VALU forms are kept out of every kernel
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-I", os.path.join(ROOT, "include"), "-o", out] + srcs


def build(verbose=False):
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    tmp = UBENCH_LIB + ".tmp%d" % os.getpid()
    cmd = command(tmp, [UBENCH_SRC])
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, UBENCH_LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
