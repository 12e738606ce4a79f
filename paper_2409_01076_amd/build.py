"""Compile the gfx950 HIP library ``libsmrt.so`` in-tree.

One translation unit (``csrc/smrt_api.hip``, which includes the kernels) is
compiled by hipcc for gfx950 only.  Packed-FP32 instructions are disabled on
purpose (``-packed-fp32-ops``): the kernels are bandwidth-bound and gain
nothing from them.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "smrt_api.hip")
LIB = os.path.join(HERE, "libsmrt.so")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
]


def build(verbose: bool = False, extra=()) -> str:
    """Compile the library; returns its path.  Always recompiles."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, *FLAGS, *extra, SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
