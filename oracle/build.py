"""Compile the C oracle into ``oracle/liboracle.so`` with gcc (plain -O2, no
fast-math, no OpenMP).  Test infrastructure only."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(force=True):
    if not force and os.path.exists(LIB):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-fPIC", "-shared",
           os.path.join(HERE, "oracle.c"), "-lm", "-o", tmp]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
