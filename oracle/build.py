"""Compile the CPU oracle (plain C) into oracle/liboracle.so.

Flags: IEEE binary32/64 in source order, no contraction, no fast-math, and
-Werror=double-promotion so that no binary32 expression is silently
evaluated in binary64.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose=False):
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
           "-Wall", "-Wextra", "-Wno-unused-parameter", "-Werror=double-promotion",
           "-o", LIB + ".tmp", os.path.join(HERE, "oracle.c"), "-lm", "-lpthread"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
