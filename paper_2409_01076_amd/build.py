"""Compile the gfx950 HIP library ``libsmrt.so`` in-tree.

Three translation units (``csrc/smrt_api.hip``: single lattices;
``csrc/smrt_batch.hip``: cavity batches; ``csrc/smrt_mlp.hip``: the warm-start
network) are compiled by hipcc for gfx950 only, in parallel, and linked into
one shared library.  Packed-FP32 instructions are disabled
(``-packed-fp32-ops``), so all FP32 arithmetic runs as one-lane-per-value
vector operations.
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
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
]


def build(verbose: bool = False, extra=()) -> str:
    """Compile the library; returns its path.  Always recompiles."""
    tag = ".tmp%d" % os.getpid()
    objs = [os.path.join(HERE, os.path.basename(src) + tag + ".o") for src in SRCS]
    try:
        procs = []
        for src, obj in zip(SRCS, objs):
            cmd = [HIPCC, *FLAGS, *extra, "-c", src, "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((cmd, subprocess.Popen(cmd)))
        failed = [cmd for cmd, p in procs if p.wait() != 0]
        if failed:
            raise subprocess.CalledProcessError(1, failed[0])
        tmp = LIB + tag
        cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    finally:
        for obj in objs:
            if os.path.exists(obj):
                os.remove(obj)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
