"""The oracle's timing build (the same source compiled with OpenMP, per-cell
and per-face loops on all host threads) computes the same bits as the
sequential parity reference: states, accumulators, levels and every
counter, for first and second order, walls and transmissive boundaries,
the predictor/corrector form and a moving mesh.  Only then may its time
stand beside the GPU's as a CPU baseline."""
import os

import numpy as np
import pytest

from paper_1704_01144_amd import inputs as I


def _run(orc, variant, nodes, tets, prim, prm, chunks, vel=None):
    orc.select(variant)
    try:
        m = orc.Mesh(nodes, tets)
        o = orc.State(m, prim, prm)
        if vel is not None:
            o.motion(vel)
        out = []
        for n in chunks:
            o.advance(n)
            out.append(o.read())
        return out, o.stats(), orc.threads()
    finally:
        orc.select("seq")


CASES = {
    "order1-walls": (lambda: I.config_small(), dict(max_levels=3, order=1), [3, 5], False),
    "order2-walls": (lambda: dict(zip(("nodes", "tets"), I.graded_cube_mesh(8, 16.0))),
                     dict(max_levels=5, order=2), [7, 9], False),
    "order2-transmissive": (lambda: dict(zip(("nodes", "tets"), I.graded_box_mesh(9, 5, 4, 4.0))),
                            dict(max_levels=4, order=2, boundary=1), [6], False),
    "time-order-2": (lambda: dict(zip(("nodes", "tets"), I.graded_cube_mesh(6, 8.0))),
                     dict(max_levels=4, order=2, time_order=2), [8, 8], False),
    "moving": (lambda: dict(zip(("nodes", "tets"), I.graded_cube_mesh(6, 4.0))),
               dict(max_levels=3, order=2), [5, 6], True),
}


@pytest.mark.parametrize("name", list(CASES))
def test_openmp_build_same_bits(orc, name):
    os.environ.setdefault("OMP_NUM_THREADS", "4")
    make, kw, chunks, moving = CASES[name]
    cfg = make()
    nodes, tets = cfg["nodes"], cfg["tets"]
    prim = cfg.get("prim")
    if prim is None:
        prim = I.blast_state(nodes, tets, centre=I.blast_centre(7))
    vel = I.motion_field(nodes, 0.05, seed=3) if moving else None
    prm = orc.params(**kw)
    seq, st_seq, n_seq = _run(orc, "seq", nodes, tets, prim, prm, chunks, vel)
    omp, st_omp, n_omp = _run(orc, "omp", nodes, tets, prim, prm, chunks, vel)
    assert n_seq == 1 and n_omp > 1
    for (u1, r1, l1), (u2, r2, l2) in zip(seq, omp):
        assert np.array_equal(u1, u2) and np.array_equal(r1, r2) and np.array_equal(l1, l2)
    assert st_seq == st_omp
