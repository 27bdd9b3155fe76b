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


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-Wno-unused-parameter",
           "-o", LIB + ".tmp"] + SRCS + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
