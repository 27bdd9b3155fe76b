"""Build the FP64 CPU oracle (test infrastructure) as a shared library: the
LB oracle (lbpf_oracle.c) and the independent finite-difference
discretisation it is checked against (fd_oracle.c).

Usage: python -m oracle.build   (or oracle.build.build() from Python)
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "lbpf_oracle.c"), os.path.join(HERE, "fd_oracle.c")]
LIB = os.path.join(HERE, "liblbpf_oracle.so")
# The LB oracle's algorithm rounded to single precision (lbpf_oracle_f32.c:
# the same source with every double and every floating constant in float;
# math-library calls still return a double, rounded once to float on
# assignment).  Test evidence of
# what FP32 state and arithmetic cost the method by themselves; never the
# reference of a comparison.
LIB_F32 = os.path.join(HERE, "liblbpf_oracle_f32.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-Wno-unused-parameter",
           "-o", LIB + ".tmp"] + SRCS + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unused-parameter",
           "-fsingle-precision-constant", "-ffp-contract=off",
           "-o", LIB_F32 + ".tmp", os.path.join(HERE, "lbpf_oracle_f32.c"), "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB_F32 + ".tmp", LIB_F32)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
