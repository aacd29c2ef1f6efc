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


# Checked build for the sanitizer test: AddressSanitizer (out-of-bounds and
# use-after-free accesses) and UndefinedBehaviorSanitizer (overflow, bad
# shifts, misaligned or null accesses), every finding fatal.
SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def build(verbose=False):
    cmd = ["gcc", *CFLAGS, SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def build_sanitized(out):
    """The oracle with SAN_FLAGS into `out` (a path outside the package)."""
    flags = [f for f in CFLAGS if f != "-O2"] + SAN_FLAGS
    subprocess.run(["gcc", *flags, SRC, "-o", out, "-lm"], check=True)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
