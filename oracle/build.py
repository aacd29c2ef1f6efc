"""Build the C oracle into oracle/liborc.so (gcc, FP64, no contraction, no fast-math).

Test infrastructure: the oracle is only ever loaded by tests/, by
__graft_entry__.smoke() and by bench.py's cpu_baseline leg.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mstar_oracle.c")
LIB = os.path.join(HERE, "liborc.so")
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
          "-Wall", "-Wextra"]


def build(verbose=False):
    cmd = ["gcc", *CFLAGS, SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
