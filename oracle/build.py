"""Build the FP64 CPU oracle library (test infrastructure).

Plain gcc, OpenMP, no FP contraction and no fast-math, so every double
operation in the oracle rounds exactly as written in the C source.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gjp_oracle.c")
LIB = os.path.join(HERE, "libgjp_oracle.so")


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = [
        "gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
        "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
        # keep sin and cos as separate libm calls (no merge into sincos, which can
        # round differently in the last bit)
        "-fno-builtin-sin", "-fno-builtin-cos", "-fno-builtin-sincos",
        SRC, "-o", tmp, "-lm",
    ]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--lazy" not in sys.argv))
