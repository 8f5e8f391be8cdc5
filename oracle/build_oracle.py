"""Compile the oracle's plain-C sweep into oracle/liboracle_sweep.so (test infrastructure)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sweep.c")
LIB = os.path.join(HERE, "liboracle_sweep.so")


def build(force=True):
    """gcc -O2 (no fast-math, no vectorisation flags beyond -O2) -> shared object."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c99", "-o", tmp, SRC, "-lm"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
