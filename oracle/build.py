"""Build the FP64 CPU oracle (test infrastructure) into oracle/_build/libvista_oracle.so.

Flags: -O3 -march=native for speed, -ffp-contract=off and no fast-math so the index and
table arithmetic follows the written operation sequence exactly, -fopenmp for the
rest-channel slabs.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "vista_oracle.c")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "libvista_oracle.so")


def build(verbose: bool = False, portable_simd: bool = True) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=c11", "-O3", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter", SRC, "-o", tmp, "-lm"]
    if portable_simd:  # the library travels to hosts of another CPU family
        cmd.insert(3, "-march=x86-64-v2")
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
