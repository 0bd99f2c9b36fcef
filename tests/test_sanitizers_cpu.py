"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

The oracle (oracle/oracle.c) and the library's host mesh preparation
(csrc/mesh_prep.cpp) are built with -fsanitize=address,undefined into small
driver programs (tests/native/), which run them on a graded blast mesh in
several configurations; any sanitizer report fails the run.  The drivers'
results are compared with the regular builds: the oracle's final states and
counters bit for bit (no FMA contraction on this host, so the optimisation
level does not change the arithmetic), the mesh preparation against what
tafv_mesh_inspect reports.  No GPU is involved.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_1704_01144_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]
ROCM_CLANG = "/opt/rocm/llvm/bin/clang++"


@pytest.fixture(scope="module")
def T():
    from paper_1704_01144_amd import tafv
    return tafv


def _san_env():
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:exitcode=86"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1:exitcode=87"
    return env


def _case():
    nodes, tets = I.graded_box_mesh(6, 5, 4, 4.0)
    prim = I.blast_state(nodes, tets, centre=I.blast_centre(4))
    vel = I.motion_field(nodes, 0.05, seed=1)
    return nodes, tets, prim, vel


def _write_input(path, nodes, tets, prim, vel):
    with open(path, "wb") as f:
        np.array([len(nodes), len(tets)], np.int64).tofile(f)
        np.ascontiguousarray(nodes, np.float64).tofile(f)
        np.ascontiguousarray(tets, np.int64).tofile(f)
        np.ascontiguousarray(prim, np.float64).tofile(f)
        np.ascontiguousarray(vel, np.float64).tofile(f)


def _run(exe, inp, out):
    r = subprocess.run([exe, inp, out], capture_output=True, text=True, env=_san_env(),
                       timeout=300)
    assert r.returncode == 0, f"{os.path.basename(exe)} exited {r.returncode}:\n{r.stderr[-4000:]}"
    assert "runtime error" not in r.stderr, r.stderr[-4000:]


# order, time order, boundary, max levels, moving, the two advance calls
CONFIGS = [(1, 1, 0, 3, False, 4, 3), (2, 1, 0, 4, False, 8, 5), (2, 1, 1, 3, False, 6, 2),
           (2, 2, 0, 3, False, 8, 4), (2, 1, 0, 3, True, 6, 2)]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is not installed")
def test_oracle_under_sanitizers(tmp_path, orc):
    exe = str(tmp_path / "oracle_check")
    subprocess.run(["gcc", "-std=c99", *SAN, "-I", os.path.join(ROOT, "oracle"),
                    os.path.join(NATIVE, "oracle_check.c"), os.path.join(ROOT, "oracle", "oracle.c"),
                    "-lm", "-o", exe], check=True)
    nodes, tets, prim, vel = _case()
    inp, out = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    _write_input(inp, nodes, tets, prim, vel)
    _run(exe, inp, out)
    raw = np.fromfile(out, np.uint8)
    n = len(tets)
    rec = 5 * n * 8 + 16
    assert raw.size == rec * len(CONFIGS)
    mesh = orc.Mesh(nodes, tets)
    for k, (order, to, bc, L, moving, n1, n2) in enumerate(CONFIGS):
        chunk = raw[k * rec:(k + 1) * rec]
        cons = chunk[:5 * n * 8].view(np.float64).reshape(n, 5)
        cells, newton = chunk[5 * n * 8:].view(np.int64)
        s = orc.State(mesh, prim, orc.params(max_levels=L, order=order, boundary=bc,
                                              time_order=to))
        if moving:
            s.motion(vel)
        s.advance(n1)
        s.advance(n2)
        ref, _, _ = s.read()
        st = s.stats()
        assert np.array_equal(cons, ref), k
        assert (cells, newton) == (st["cell_updates"], st["newton_updates"]), k


@pytest.mark.skipif(not os.path.exists(ROCM_CLANG), reason="the ROCm clang is not installed")
def test_mesh_preparation_under_sanitizers(tmp_path, T):
    exe = str(tmp_path / "mesh_prep_check")
    csrc = os.path.join(ROOT, "paper_1704_01144_amd", "csrc")
    subprocess.run([ROCM_CLANG, "-std=c++17", "-x", "c++", *SAN, "-D__HIP_PLATFORM_AMD__",
                    "-I/opt/rocm/include", "-I", os.path.join(ROOT, "include"), "-I", csrc,
                    os.path.join(NATIVE, "mesh_prep_check.cpp"),
                    os.path.join(csrc, "mesh_prep.cpp"), "-o", exe], check=True)
    nodes, tets, prim, vel = _case()
    inp, out = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    _write_input(inp, nodes, tets, prim, vel)
    _run(exe, inp, out)
    raw = np.fromfile(out, np.uint8)
    nf, nbnd, ncol = raw[:24].view(np.int64)
    ref = T.tafv_mesh_inspect(nodes, tets)
    assert (nf, nbnd, ncol) == (ref["n_faces"], ref["n_boundary"], ref["n_colours"])
    o = 24
    col = raw[o:o + nf].view(np.int8)
    o += nf
    area = raw[o:o + 24 * nf].view(np.float64).reshape(nf, 3)
    o += 24 * nf
    nb = raw[o:o + 16 * len(tets)].view(np.int32).reshape(len(tets), 4)
    assert o + 16 * len(tets) == raw.size
    assert np.array_equal(col, ref["face_colour"])
    assert np.array_equal(area, ref["face_area"])
    assert np.array_equal(np.where(nb >= 0, nb, -1), ref["cell_neighbours"])
