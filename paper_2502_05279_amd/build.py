"""Build the HIP library ``libbmg.so`` for gfx950, in-tree.

    python -m paper_2502_05279_amd.build

FP contraction is off (``-ffp-contract=off``) so that every product and sum
is rounded as written, and packed FP32 instructions are disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "lib")
LIB = os.path.join(OUT_DIR, "libbmg.so")
ARCH = os.environ.get("BMG_OFFLOAD_ARCH", "gfx950")

SOURCES = ["bmg_runtime.hip", "bmg_batch.hip", "bmg_learn.hip", "bmg_nonsym.hip"]
HEADERS = [os.path.join(ROOT, "include", "bmg.h")]


def _deps():
    out = [os.path.join(CSRC, f) for f in os.listdir(CSRC)] + HEADERS
    return [p for p in out if os.path.isfile(p)]


def command(out: str, defines=()) -> list[str]:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    return [hipcc, f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
            *[f"-D{d}" for d in defines],
            "-ffp-contract=off", "-fno-fast-math",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC,
            *[os.path.join(CSRC, s) for s in SOURCES], "-o", out]


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    """Compiles the library to ``out`` (with extra -D definitions, e.g. a
    tuning variant such as BMG_FIVE_POINT_STEP_ROWS=4)."""
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp"
    cmd = command(tmp, defines)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def needs_build() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in _deps())


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
