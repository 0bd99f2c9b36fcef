"""Pins of the oracle's predictor/corrector form of the temporal-adaptive
scheme (Sec. 2.2, Alg. 2: predictor, prediction, interpolation of the
slower levels, corrector, correction), time_order = 2.

  * one level: the predictor/corrector step is Heun's method, which equals
    the Shu-Osher form (U + FE(FE(U))) / 2 built from two forward Euler
    steps of the pinned first-order scheme;
  * several levels: the error at a fixed final time against a global
    fine-step solution falls by 4 when the time steps halve (second order in
    time), where the forward Euler form falls by 2 -- and a copy of the
    scheme without the interpolation of slower neighbours falls by 2 too,
    so the test sees that interpolation;
  * conservation of mass and energy (and momentum up to the wall impulse)
    after every subiteration, counting the pending accumulators;
  * free-stream preservation across levels.
"""
import numpy as np
import pytest

from paper_1704_01144_amd import inputs as I


def _run(orc, m, prim, time_order, cfl, L, iterations, order=1, boundary=0):
    """`iterations` whole iterations with the first classification kept
    (fixed levels and dt_min, so runs at cfl and cfl/2 end at the same time)."""
    st = orc.State(m, prim, orc.params(max_levels=L, order=order, reclassify=0,
                                       time_order=time_order, cfl=cfl, boundary=boundary))
    st.advance(1)
    theta = st.stats()["theta"]
    st.advance(iterations * 2 ** theta - 1)
    return st


@pytest.mark.parametrize("order", [1, 2])
def test_single_level_is_heun_shu_osher(orc, order):
    nodes, tets = I.graded_box_mesh(5, 5, 5, 3.0)
    m = orc.Mesh(nodes, tets)
    prim = I.blast_state(nodes, tets, centre=(0.4, 0.5, 0.6), radius=0.3, p_in=3.0)
    u0 = orc.prim_to_cons(prim)
    heun = orc.State(m, prim, orc.params(max_levels=1, order=order, reclassify=0, time_order=2))
    heun.advance(1)
    uh = heun.read()[0]
    fe = orc.State(m, prim, orc.params(max_levels=1, order=order, reclassify=0))
    fe.advance(1)
    u1, _, lev = fe.read()
    s = fe.stats()
    fe.set(u1, np.zeros_like(u1), lev, 0, 0, s["dt_min"], s["t_reached"])
    fe.advance(1)
    u2 = fe.read()[0]
    expect = 0.5 * (u0 + u2)
    assert heun.stats()["dt_min"] == s["dt_min"]
    assert np.abs(uh - expect).max() < 1e-13 * np.abs(uh - u0).max() + 1e-15
    # two solves per face: predictor and corrector
    assert heun.stats()["face_solves"] == 2 * m.n_faces


def _errors(orc, m, prim, time_order, L, order, cfl=0.4, iterations=2):
    probe = _run(orc, m, prim, 2, cfl, L, 1, order)
    theta = probe.stats()["theta"]
    ref = orc.State(m, prim, orc.params(max_levels=1, order=order, reclassify=0, time_order=2,
                                        cfl=cfl / 32))
    ref.advance(32 * iterations * 2 ** theta)
    u_ref, t_ref = ref.read()[0], ref.stats()["t_reached"]
    errs = []
    for k in (1, 2, 4):
        st = _run(orc, m, prim, time_order, cfl / k, L, iterations * k, order)
        assert abs(st.stats()["t_reached"] - t_ref) <= 1e-12 * t_ref
        errs.append(np.abs(st.read()[0] - u_ref).max())
    return theta, np.array(probe.stats()["cells_per_level"]), errs


@pytest.mark.parametrize("order", [1, 2])
def test_second_order_in_time_across_levels(orc, order):
    nodes, tets = I.graded_box_mesh(6, 6, 6, 16.0)
    m = orc.Mesh(nodes, tets)
    prim = I.pulse_state(nodes, tets)
    theta, hist, e2 = _errors(orc, m, prim, 2, 4, order)
    assert theta == 3 and (hist[:4] > 0).all()  # four levels in use
    r2 = [e2[0] / e2[1], e2[1] / e2[2]]
    assert min(r2) > 3.6, r2
    _, _, e1 = _errors(orc, m, prim, 1, 4, order)
    r1 = [e1[0] / e1[1], e1[1] / e1[2]]
    assert max(r1) < 2.4, r1
    assert e2[2] < 0.05 * e1[2]


@pytest.mark.parametrize("order", [1, 2])
def test_conservation_every_subiteration(orc, order):
    nodes, tets = I.graded_cube_mesh(8, 4.0)
    m = orc.Mesh(nodes, tets)
    prim = I.blast_state(nodes, tets, centre=(0.3, 0.6, 0.5))
    prim[:, 1:4] = np.random.default_rng(1).uniform(-0.4, 0.4, (len(prim), 3))
    vol = m.geometry()["vol"][:, None]
    st = orc.State(m, prim, orc.params(max_levels=4, order=order, time_order=2))
    tot0 = (vol * orc.prim_to_cons(prim)).sum(0)
    mid = 0
    for k in range(19):
        st.advance(1)
        u, r, lev = st.read()
        tot = (vol * u).sum(0) + r.sum(0)
        s = st.stats()
        for c in (0, 4):
            assert abs(tot[c] - tot0[c]) < 1e-13 * abs(tot0[c])
        mom = tot[1:4] + np.array(s["wall_impulse"])
        scale = (vol * np.abs(u[:, 1:4])).sum() + np.abs(s["wall_impulse"]).sum() + (vol * u[:, :1]).sum()
        assert np.abs(mom - tot0[1:4]).max() < 1e-13 * scale
        mid += s["phase"] != 0 and np.abs(r).max() > 0  # checked with pending sums
    assert s["theta"] >= 2 and mid > 5
    st.advance(2 ** s["theta"] - s["phase"])
    assert (st.read()[1] == 0).all()


def test_free_stream_preserved(orc):
    nodes, tets = I.graded_cube_mesh(6, 4.0)
    m = orc.Mesh(nodes, tets)
    prim = np.tile([1.2, 0.3, -0.2, 0.1, 0.9], (len(tets), 1))
    st = orc.State(m, prim, orc.params(max_levels=3, order=2, boundary=1, time_order=2))
    st.advance(8)
    u0 = orc.prim_to_cons(prim)
    assert st.stats()["theta"] >= 1
    assert np.abs(st.read()[0] - u0).max() < 1e-14 * np.abs(u0).max()


def test_checkpoint_only_at_iteration_start(orc):
    nodes, tets = I.graded_cube_mesh(3, 2.0)
    m = orc.Mesh(nodes, tets)
    prim = I.blast_state(nodes, tets)
    st = orc.State(m, prim, orc.params(max_levels=3, time_order=2))
    u, r, lev = st.read()
    with pytest.raises(orc.OracleError):
        st.set(u, r, np.ones_like(lev), 1, 1, 1e-3)
    st.set(u, r, lev, 0, 0, 1e-3)
    with pytest.raises(orc.OracleError):
        orc.State(m, prim, orc.params(time_order=3))
