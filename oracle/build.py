"""Build the FP64 oracle shared library (test infrastructure only).

gcc -O2, no fast-math: the oracle is the plain reference, never tuned.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "nsn_oracle.c")
HDR = os.path.join(HERE, "nsn_oracle.h")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose=False, src=SRC, out=LIB):
    """Compile the oracle (or a variant source `src`, e.g. one with a planted mistake,
    into `out`)."""
    cmd = ["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-Wall", "-fPIC", "-shared",
           "-I", HERE, "-o", out + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
