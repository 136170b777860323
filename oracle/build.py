"""Builds the oracle's shared library with gcc (test infrastructure only)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "epi3_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build_oracle(src: str = SRC, out: str = LIB, extra=()) -> str:
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-Wall",
           *extra, src, "-o", out, "-lm"]
    subprocess.run(cmd, check=True)
    return out


if __name__ == "__main__":
    print(build_oracle(*sys.argv[1:2]))
