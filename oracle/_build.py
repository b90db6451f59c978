"""Build step for the oracle's shared library (plain C, gcc, FP64, no FMA
contraction, no fast-math; OpenMP splits independent cells only)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def library_path():
    return os.path.join(HERE, "liboracle.so")


def build(verbose=False):
    src = os.path.join(HERE, "gbr_oracle.c")
    out = library_path()
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared", "-std=c99", "-Wall", "-Wextra", "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
