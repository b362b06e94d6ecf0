"""Build step for the FP64 CPU oracle (test infrastructure only).

Compiles ``prenom_oracle.c`` with gcc into ``liboracle.so`` next to this file:
no fast-math and no floating-point contraction, so every FP64 expression is
evaluated exactly as written; OpenMP parallelises per-ray work only.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "prenom_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

CFLAGS = [
    "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
    "-fno-fast-math", "-ffp-contract=off", "-fno-finite-math-only",
    "-Wall", "-Wextra", "-Wno-unused-parameter",
]


def build_oracle(verbose: bool = False) -> str:
    """Compile the oracle library and return its path."""
    tmp = LIB + ".tmp"
    cmd = ["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_oracle(verbose=True))
