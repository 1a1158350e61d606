"""Builds the CPU oracle library (test infrastructure only).

The oracle is plain C compiled with gcc.  -ffp-contract=off keeps every
multiply and add a separately rounded operation (no FMA contraction), and no
-ffast-math flag is given, so division by 6 is IEEE division.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = [os.path.join(HERE, "oracle.c"), os.path.join(HERE, "lbm.c")]
LIB = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
          "-fPIC", "-shared", "-Wall", "-Wextra"]


def build(verbose=False):
    """Compile oracle.c and lbm.c into liboracle.so next to them; returns the
    library path."""
    cmd = ["gcc", *CFLAGS, *SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
