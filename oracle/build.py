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


LIB_F32 = os.path.join(HERE, "liboracle_f32.so")


def build(verbose=False, src=SRC, out=LIB, extra=()):
    """Compile the oracle (or a variant source `src`, e.g. one with a planted mistake,
    into `out`; `extra`: more compiler flags)."""
    cmd = ["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-Wall", "-fPIC", "-shared",
           "-I", HERE] + list(extra) + ["-o", out + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def build_f32(verbose=False):
    """The same source with every double replaced by float (API included): the
    algorithm evaluated in single precision.  A test probe, not an oracle: the per-row
    parity tests use its distance from the FP64 build as an estimate of what FP32
    rounding alone does to each quantity (cancellation included)."""
    return build(verbose=verbose, src=os.path.join(HERE, "nsn_oracle_f32.c"), out=LIB_F32)


if __name__ == "__main__":
    build(verbose=True)
    build_f32(verbose=True)
    sys.exit(0)
