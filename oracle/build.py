"""Compile the oracle's C code (test infrastructure only).

Builds ``oracle/libknn_brute.so`` with gcc and OpenMP.  No -ffast-math and no
host-specific ISA flags: the sums keep their written order, and the library
runs on any x86-64 host.
"""
from __future__ import annotations

import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))


def build(verbose: bool = False) -> str:
    src = os.path.join(_HERE, "knn_brute.c")
    out = os.path.join(_HERE, "libknn_brute.so")
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
