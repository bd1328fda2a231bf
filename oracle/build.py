"""Builds the CPU oracle's C library (liboracle_ref.so) with gcc.

Test infrastructure only: the tests, the package smoke check and the
benchmark's CPU-baseline leg are the only users.  -ffp-contract=off keeps
the compiler from fusing anything beyond the fma() calls the source makes.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ref.c")
LIB = os.path.join(HERE, "liboracle_ref.so")


def build(force=False):
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-std=gnu11", "-O2", "-fPIC", "-shared",
                           "-ffp-contract=off", "-fno-fast-math", "-o", tmp, SRC, "-lm"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True))
