"""Build the CPU oracle shared library (test infrastructure only).

    python -m oracle.build      # writes oracle/liborc.so
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "af_oracle.cpp")
LIB = os.path.join(HERE, "liborc.so")

# Plain IEEE double: no fast-math, no FMA contraction.
FLAGS = ["-O2", "-std=c++17", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math"]


def build(verbose: bool = False) -> str:
    cmd = ["g++", *FLAGS, SRC, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
