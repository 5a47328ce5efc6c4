"""Build the oracle's C library (test infrastructure only).

Compiles ``oracle/gemm_ref.c`` into ``oracle/libgemm_ref.so`` with gcc.  The
flags keep the arithmetic plain: no FMA contraction (``-ffp-contract=off``), so
every product and sum is a separately rounded IEEE double operation, and a
portable x86-64-v3 target so the library built here also runs on the GPU
host's CPU.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gemm_ref.c")
LIB = os.path.join(HERE, "libgemm_ref.so")

CFLAGS = ["-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fopenmp",
          "-fPIC", "-shared", "-std=c11"]


def build(force: bool = True) -> str:
    """Compile the oracle library; returns its path."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    subprocess.run(["gcc", *CFLAGS, SRC, "-o", tmp], check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
