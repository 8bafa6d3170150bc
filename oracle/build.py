"""Build the CPU oracle shared library (test infrastructure only).

    python -m oracle.build      # writes oracle/liborc.so
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "af_oracle.cpp")
LIB = os.path.join(HERE, "liborc.so")
LIB_SAN = os.path.join(HERE, "liborc_san.so")

# Plain IEEE double: no fast-math, no FMA contraction.
FLAGS = ["-O2", "-std=c++17", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math"]
# The same with address and undefined-behaviour sanitizers (a checked build that the
# oracle's pins can run against; see tests/test_sanitize.py).
SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def build(verbose: bool = False, sanitize: bool = False) -> str:
    out = LIB_SAN if sanitize else LIB
    flags = [f for f in FLAGS if not (sanitize and f == "-O2")] + (SAN_FLAGS if sanitize else [])
    cmd = ["g++", *flags, SRC, "-o", out + ".tmp"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
