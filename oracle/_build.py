"""Compiles the oracle's C source into ``oracle/liboracle.so`` with gcc.

Test infrastructure only (see ``oracle/__init__.py``).  Flags: ``-O3
-fopenmp`` at the x86-64-v3 level (AVX2 + FMA), the survey's timing
protocol except for ``-march=native``: the built library also runs on other
hosts than the one that built it, whose CPUs may lack this host's newest
instructions.  The source is the oracle as written, not tuned for speed.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "direct.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
