"""Builds the generator's C fast path (libdsrgen.so) with gcc."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fastgen.c")
LIB = os.path.join(HERE, "libdsrgen.so")


def build(force=False):
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-std=gnu11", "-O2", "-fPIC", "-shared", "-pthread", "-o", tmp, SRC])
    os.replace(tmp, LIB)
    return LIB
