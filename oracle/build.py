"""Build the oracle shared library (test infrastructure).

Plain gcc, FP64, no contraction of multiply-adds, so the oracle's rounding is
that of the source as written.  A second build of the same source with
multiply-adds contracted into fused ones (liboracle_fma.so) only measures the
oracle's sensitivity to rounding: the difference between the two builds after
a long run is what a correct implementation that rounds differently (as a GPU
compiler's contraction does) can leave.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rmhdlb_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
LIB_FMA = os.path.join(HERE, "liboracle_fma.so")


def build(verbose: bool = False, fma: bool = False) -> str:
    out = LIB_FMA if fma else LIB
    contract = ["-ffp-contract=fast", "-mfma"] if fma else ["-ffp-contract=off"]
    cmd = ["gcc", "-O2"] + contract + ["-fno-fast-math", "-fPIC", "-shared", "-std=c11",
                                       "-Wall", "-Wextra", "-o", out + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
