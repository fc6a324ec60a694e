"""Build step for the oracle's C part (test infrastructure only).

Compiles ``pairderiv.c`` into ``liboracle.so`` beside it with plain gcc,
``-O2 -ffp-contract=off`` (no fused multiply-adds, no fast-math) and OpenMP.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pairderiv.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(force=True):
    """Compile the oracle library; with ``force=False`` only if it is missing or stale."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared", "-std=c99", "-Wall", "-Wno-maybe-uninitialized", "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
