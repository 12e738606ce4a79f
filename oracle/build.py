"""Compile the FP64 CPU oracle into ``oracle/libsmrt_oracle.so``.

Test infrastructure only: the oracle checks the GPU library and is never part
of it.  Built with gcc, OpenMP, and ``-ffp-contract=off`` so that no fused
multiply-add changes the rounding of the literal formulas.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "smrt_oracle.c")
LIB = os.path.join(HERE, "libsmrt_oracle.so")

CFLAGS = ["-std=c11", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
          "-Wall", "-Wextra"]


def build(verbose: bool = False) -> str:
    """Compile the oracle; returns the path of the shared library."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
