"""Build ``libtafv.so`` (the C-ABI library with the gfx950 HIP kernels) in
place with hipcc.  Used by ``__graft_entry__.build()`` and by the tests when
no library is present."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtafv.so")
SOURCES = ["mesh_prep.cpp", "kernels.hip", "mlp.hip", "batch.hip", "capi.hip"]
ARCH = os.environ.get("TAFV_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-x", "hip",
    # a * b + c is fused where one expression writes it, never across
    # statements: an inlined device function then rounds the same way in
    # every kernel that uses it
    "-ffp-contract=on",
    # packed FP32 instructions stay off: scalar/float2 code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
    "-Wall", "-Wno-unused-result",
]


def build(verbose=False):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(CSRC, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs, cmds = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        cmds.append([hipcc] + HIPCC_FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    # the translation units compile independently, a few at a time
    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", "4"))))
    with ThreadPoolExecutor(jobs) as pool:
        for cmd in cmds:
            if verbose:
                print(" ".join(cmd), flush=True)
        for rc, cmd in zip(pool.map(subprocess.call, cmds), cmds):
            if rc != 0:
                raise subprocess.CalledProcessError(rc, cmd)
    tmp = LIB + ".tmp"
    cmd = [hipcc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
