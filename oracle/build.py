"""Compile the C oracle with gcc (plain -O2, no fast-math).

  oracle/liboracle.so      sequential: the parity reference of the tests;
  oracle/liboracle_omp.so  the same source with -fopenmp: its per-cell and
                           per-face loops run on all host threads, with the
                           same bits (timing of the CPU baseline only).

Test infrastructure only."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")


def build(force=True, openmp=False):
    lib = LIB_OMP if openmp else LIB
    if not force and os.path.exists(lib):
        return lib
    tmp = lib + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-fPIC", "-shared"]
    if openmp:
        cmd.append("-fopenmp")
    cmd += [os.path.join(HERE, "oracle.c"), "-lm", "-o", tmp]
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    return lib


def build_all(force=True):
    return build(force), build(force, openmp=True)


if __name__ == "__main__":
    print(build_all())
