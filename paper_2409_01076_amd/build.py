"""Compile the gfx950 HIP library ``libsmrt.so`` in-tree.

Three translation units (``csrc/smrt_api.hip``: single lattices;
``csrc/smrt_batch.hip``: cavity batches; ``csrc/smrt_mlp.hip``: the warm-start
network) are compiled by hipcc for gfx950 only and linked into one shared
library.  Packed-FP32 instructions are disabled on
purpose (``-packed-fp32-ops``): the kernels are bandwidth-bound and gain
nothing from them.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRCS = [os.path.join(HERE, "csrc", f) for f in ("smrt_api.hip", "smrt_batch.hip", "smrt_mlp.hip")]
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
    cmd = [HIPCC, *FLAGS, *extra, *SRCS, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
