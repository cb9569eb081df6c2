"""Build the C tier of the CPU oracle (test infrastructure only).

    python oracle/build.py

compiles ``bmg_oracle.c`` (which includes the precision-generic core and the
nonsymmetric part) with gcc, FP contraction off (so that every product
and sum is rounded exactly as written), OpenMP inside each colour / loop.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "liboracle.so")
SOURCES = ["bmg_oracle.c", "bmg_oracle_core.inc", "bmg_oracle_ns.c"]


def build(verbose: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O3", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wno-unknown-pragmas",
           os.path.join(HERE, "bmg_oracle.c"), "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def needs_build() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(os.path.join(HERE, s)) > t for s in SOURCES)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
