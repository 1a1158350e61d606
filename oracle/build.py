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


def build_sanitized(verbose=False):
    """oracle.c and lbm.c with AddressSanitizer and UndefinedBehaviorSanitizer
    (gcc), at _build/san/liboracle.so; load it into a process that preloads
    gcc's libasan and libubsan (sanitizer_runtimes())."""
    out_dir = os.path.join(os.path.dirname(HERE), "_build", "san")
    os.makedirs(out_dir, exist_ok=True)
    out = os.path.join(out_dir, "liboracle.so")
    flags = [f for f in CFLAGS if f != "-O2"] + ["-O1", "-g", "-fsanitize=address,undefined",
                                                 "-fno-sanitize-recover=undefined",
                                                 "-fno-omit-frame-pointer"]
    cmd = ["gcc", *flags, *SRC, "-o", out, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return out


def sanitizer_runtimes():
    """gcc's shared libasan and libubsan (to preload, in that order)."""
    out = []
    for name in ("libasan.so", "libubsan.so"):
        path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True,
                              text=True).stdout.strip()
        if not os.path.isabs(path):
            raise FileNotFoundError(name)
        out.append(os.path.realpath(path))
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
