"""Pins of the oracle's moving-mesh form (Sec. 2.1: an ALE formulation in
which the face velocity enters the flux, and cell volumes that follow the
geometric conservation law; the face geometry stays that of the uploaded
mesh, the form used for slow relative motion).

  * the moving-face flux is the fixed-face flux of the Galilean-shifted
    face problem, transformed back (momentum + xi n F_mass, energy +
    xi n . F_mom + xi^2/2 F_mass), for interior, wall and transmissive
    faces; xi = 0 gives the fixed-face flux;
  * geometric conservation: a uniform state stays uniform under any node
    motion, over several levels, at second order;
  * an affine node velocity v(x) = B x changes every cell's volume at the
    rate tr(B) V (divergence theorem, exact for linear fields);
  * a uniform translation of the whole mesh (walls included) with velocity
    c gives the fixed-mesh solution of the state with velocity u - c, with
    identical levels (Galilean invariance of the Euler equations);
  * mass, momentum (with the wall impulse), energy and total volume are
    conserved at every subiteration when only interior nodes move.
"""
import numpy as np
import pytest

from paper_1704_01144_amd import inputs as I


def _boundary_nodes(m, tets):
    g = m.geometry()
    cf, fR = g["cell_faces"], g["face_R"]
    tets = np.asarray(tets)
    out = set()
    for j in range(4):
        on = fR[cf[:, j]] < 0
        for k in range(4):
            if k != j:
                out.update(tets[on, k].tolist())
    return np.array(sorted(out))


def test_moving_face_flux_is_shifted_fixed_flux(orc):
    rng = np.random.default_rng(0)
    worst = 0.0
    for _ in range(300):
        wl = np.array([rng.uniform(0.3, 3), *rng.uniform(-1.5, 1.5, 3), rng.uniform(0.2, 4)])
        wr = np.array([rng.uniform(0.3, 3), *rng.uniform(-1.5, 1.5, 3), rng.uniform(0.2, 4)])
        A = rng.normal(size=3)
        n = A / np.linalg.norm(A)
        xi = rng.uniform(-1.0, 1.0)
        for kind in (orc.KIND_INTERIOR, orc.KIND_WALL, orc.KIND_TRANSMIT):
            fm, _ = orc.face_flux_moving(wl, wr, A, xi, kind)
            sl, sr = wl.copy(), wr.copy()
            sl[1:4] -= xi * n
            sr[1:4] -= xi * n
            fs, _ = orc.face_flux(sl, sr, A, kind)
            exp = fs.copy()
            exp[1:4] = fs[1:4] + xi * n * fs[0]
            exp[4] = fs[4] + xi * (n @ fs[1:4]) + 0.5 * xi * xi * fs[0]
            worst = max(worst, np.abs(fm - exp).max() / np.abs(exp).max())
        f0, _ = orc.face_flux_moving(wl, wr, A, 0.0)
        f1, _ = orc.face_flux(wl, wr, A)
        assert np.abs(f0 - f1).max() <= 1e-14 * np.abs(f1).max()
    assert worst < 1e-13


@pytest.mark.parametrize("order", [1, 2])
def test_uniform_state_stays_uniform(orc, order):
    nodes, tets = I.graded_box_mesh(6, 5, 4, 8.0)
    m = orc.Mesh(nodes, tets)
    prim = np.tile([1.2, 0.3, -0.2, 0.1, 0.9], (len(tets), 1))
    st = orc.State(m, prim, orc.params(max_levels=3, order=order, boundary=orc.BC_TRANSMIT))
    st.motion(np.random.default_rng(1).uniform(-0.05, 0.05, (len(nodes), 3)))
    st.advance(16)
    u0 = orc.prim_to_cons(prim)
    assert st.stats()["theta"] >= 1
    assert np.abs(st.read()[0] - u0).max() < 1e-14 * np.abs(u0).max()
    assert np.abs(st.volumes() - m.geometry()["vol"]).max() > 1e-6  # the volumes did move


def test_affine_motion_volume_rate(orc):
    nodes, tets = I.graded_box_mesh(6, 5, 4, 8.0)
    m = orc.Mesh(nodes, tets)
    B = np.array([[0.1, 0.02, 0.0], [0.0, -0.05, 0.03], [0.01, 0.0, 0.2]])
    st = orc.State(m, I.blast_state(nodes, tets), orc.params(max_levels=3, order=2, reclassify=0))
    st.motion(nodes @ B.T)
    st.advance(1)
    theta = st.stats()["theta"]
    st.advance(2 * 2 ** theta - 1)
    T = st.stats()["t_reached"]
    v0 = m.geometry()["vol"]
    assert theta >= 1
    assert np.abs(st.volumes() - v0 * (1.0 + T * np.trace(B))).max() < 1e-14 * v0.max()


@pytest.mark.parametrize("order", [1, 2])
def test_translation_is_galilean(orc, order):
    nodes, tets = I.graded_box_mesh(6, 5, 4, 8.0)
    m = orc.Mesh(nodes, tets)
    rng = np.random.default_rng(2)
    c = np.array([0.3, -0.2, 0.1])
    prim = I.blast_state(nodes, tets, centre=(0.4, 0.5, 0.5))
    prim[:, 1:4] = rng.uniform(-0.2, 0.2, (len(tets), 3))
    moving = orc.State(m, prim, orc.params(max_levels=4, order=order))
    moving.motion(np.tile(c, (len(nodes), 1)))
    shifted = prim.copy()
    shifted[:, 1:4] -= c
    fixed = orc.State(m, shifted, orc.params(max_levels=4, order=order))
    moving.advance(1)
    fixed.advance(1)
    n = 2 * 2 ** moving.stats()["theta"] - 1
    moving.advance(n)
    fixed.advance(n)
    ua, _, la = moving.read()
    ub, _, lb = fixed.read()
    pa, pb = orc.cons_to_prim(ua), orc.cons_to_prim(ub)
    pa[:, 1:4] -= c
    assert moving.stats()["theta"] >= 2
    assert (la == lb).all()
    assert np.abs(pa - pb).max() < 1e-13 * np.abs(pb).max()


def test_conservation_with_interior_motion(orc):
    nodes, tets = I.graded_box_mesh(7, 6, 5, 8.0)
    m = orc.Mesh(nodes, tets)
    vel = np.random.default_rng(3).uniform(-0.05, 0.05, (len(nodes), 3))
    vel[_boundary_nodes(m, tets)] = 0.0
    prim = I.blast_state(nodes, tets, centre=(0.4, 0.5, 0.5))
    st = orc.State(m, prim, orc.params(max_levels=4, order=2))
    st.motion(vel)
    v0 = m.geometry()["vol"]
    tot0 = (v0[:, None] * orc.prim_to_cons(prim)).sum(0)
    for k in range(20):
        st.advance(1)
        u, r, lev = st.read()
        V = st.volumes()
        tot = (V[:, None] * u).sum(0) + r.sum(0)
        s = st.stats()
        for c in (0, 4):
            assert abs(tot[c] - tot0[c]) < 1e-13 * abs(tot0[c])
        mom = tot[1:4] + np.array(s["wall_impulse"])
        assert np.abs(mom - tot0[1:4]).max() < 1e-13 * tot0[0]
    assert s["theta"] >= 2
    st.advance(2 ** s["theta"] - s["phase"])
    assert abs(st.volumes().sum() - v0.sum()) < 1e-14 * v0.sum()
    assert np.abs(st.volumes() - v0).max() > 1e-6


def test_motion_rules(orc):
    nodes, tets = I.graded_cube_mesh(3, 2.0)
    m = orc.Mesh(nodes, tets)
    prim = I.blast_state(nodes, tets)
    st = orc.State(m, prim, orc.params(max_levels=3, time_order=2))
    with pytest.raises(orc.OracleError):
        st.motion(np.zeros((len(nodes), 3)))
    st = orc.State(m, prim, orc.params(max_levels=3))
    bad = np.zeros((len(nodes), 3))
    bad[0, 0] = np.nan
    with pytest.raises(orc.OracleError):
        st.motion(bad)
    st.motion(np.zeros((len(nodes), 3)))
    u, r, lev = st.read()
    with pytest.raises(orc.OracleError):
        st.set(u, r, lev, 0, 0, 1e-3)
