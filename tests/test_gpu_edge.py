"""GPU parity on the method's edge paths, against the FP64 oracle run with the
same parameters on the same seeded inputs:

  * the bisection fallback of the p* solve: with at most one Newton update
    per face, every face whose start is not already the root falls back to
    bisection (the oracle counts the same faces);
  * a ratio of specific heats other than 1.4 (5/3): the generic-power
    solver and sampler instead of the 7th-root forms;
  * Riemann problems that generate vacuum (the pressure positivity
    condition fails): the two sides' normal velocities part faster than
    their rarefactions can follow, and the sample at x/t = 0 falls in the
    vacuum, in the left fan or in the right fan.  The case was designed on
    the CPU with the oracle first: ten subiterations keep density and
    pressure positive;
  * the judge of the learned start: a network whose correction makes
    p_TR exp(y) overflow (or underflow to 0) is rejected face by face, and
    the run is bit-identical to the two-rarefaction start;
  * a non-finite network parameter is refused (TAFV_E_MLP).

Bar: the FP64 bar of the other parity tests (normwise <= 1e-12 on cons +
accum / V, with the momentum scaled as a vector; identical levels and
schedule counters), plus the fallback and vacuum counters against the
oracle's.
"""
import sys

import numpy as np
import pytest

from oracle import mlp_ref as M
from paper_1704_01144_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def T():
    from paper_1704_01144_amd import tafv
    return tafv


def normwise(a, b):
    """max_i |a_ik - b_ik| / scale_k over the components k, with the
    momentum components scaled by the largest momentum component of b (the
    momentum vector's norm): in the vacuum cases the flow is along x, and
    the y and z momenta stay at rounding level, where a per-component scale
    would compare rounding with rounding."""
    scale = np.abs(b).max(0)
    scale[1:4] = scale[1:4].max()
    scale[scale == 0] = 1.0
    return (np.abs(a - b).max(0) / scale).max()


def run_pair(T, orc, nodes, tets, prim, chunks, order, L, gamma=1.4, newton_max_iter=50,
             boundary=0, scatter=1):
    """Advance the GPU path and the oracle by the same chunks; compare after
    each chunk.  Returns the GPU and oracle counters."""
    say(f"case: cells={len(tets)} order={order} L={L} gamma={gamma:.4f} "
        f"newton_max_iter={newton_max_iter} boundary={boundary} scatter={scatter} "
        f"chunks={chunks}")
    s = T.Solver(max_levels=L, order=order, gamma=gamma, newton_max_iter=newton_max_iter,
                 boundary=boundary, scatter=scatter)
    s.upload(nodes, tets)
    s.init(prim)
    m = orc.Mesh(nodes, tets)
    vol = m.geometry()["vol"][:, None]
    o = orc.State(m, prim, orc.params(gamma=gamma, max_levels=L, order=order, boundary=boundary,
                                      newton_max_iter=newton_max_iter))
    for n in chunks:
        s.advance(n)
        o.advance(n)
        ck = s.checkpoint()
        u_o, r_o, lev_o = o.read()
        assert (ck["levels"] == lev_o).all()
        err = normwise(ck["cons"] + ck["accum"] / vol, u_o + r_o / vol)
        say(f"  after {n}: normwise err {err:.3e}")
        assert err <= TOL, err
    sg, so = s.stats(), o.stats()
    s.close()
    for k in ("subiterations", "cell_updates", "face_solves", "theta", "phase", "vacuum_faces"):
        assert sg[k] == so[k], (k, sg[k], so[k])
    assert sg["cells_per_level"] == so["cells_per_level"]
    say(f"  counters: face solves {sg['face_solves']}, Newton {sg['newton_updates']} / "
        f"{so['newton_updates']}, fallbacks {sg['newton_fallbacks']} / {so['newton_fallbacks']}, "
        f"vacuum {sg['vacuum_faces']}")
    # a face whose one Newton update lands at the stop tolerance may be
    # decided differently by the two rounding sequences
    assert abs(sg["newton_fallbacks"] - so["newton_fallbacks"]) <= 1e-3 * so["newton_fallbacks"] + 2
    assert abs(sg["newton_updates"] - so["newton_updates"]) <= 1e-3 * so["newton_updates"] + 5
    return sg, so


@pytest.mark.parametrize("scatter", [0, 1], ids=["colour", "gather"])
def test_bisection_fallback_first_order(T, orc, scatter):
    cfg = I.config_small()
    sg, so = run_pair(T, orc, cfg["nodes"], cfg["tets"], cfg["prim"], [1, 3, 4], 1,
                      cfg["max_levels"], newton_max_iter=1, scatter=scatter)
    # every face with a shock needs more than one update and falls back
    # (4.5% of the face solves of this blast; the others are at rest or in
    # rarefactions, where the two-rarefaction start is the root)
    assert so["newton_fallbacks"] > 1000


def test_bisection_fallback_second_order(T, orc):
    nodes, tets = I.graded_cube_mesh(12, 16.0)
    prim = I.blast_state(nodes, tets, centre=I.blast_centre(3))
    sg, so = run_pair(T, orc, nodes, tets, prim, [5, 11], 2, 5, newton_max_iter=1)
    assert so["newton_fallbacks"] > 1000


@pytest.mark.parametrize("order", [1, 2])
def test_gamma_five_thirds(T, orc, order):
    nodes, tets = I.graded_cube_mesh(12, 8.0)
    prim = I.blast_state(nodes, tets, centre=I.blast_centre(4))
    run_pair(T, orc, nodes, tets, prim, [3, 13], order, 4, gamma=5.0 / 3.0)


def test_gamma_five_thirds_fallback_transmissive(T, orc):
    nodes, tets = I.graded_box_mesh(10, 6, 5, 4.0)
    prim = I.blast_state(nodes, tets, centre=(0.4, 0.5, 0.5))
    sg, so = run_pair(T, orc, nodes, tets, prim, [8], 2, 3, gamma=5.0 / 3.0, newton_max_iter=2,
                      boundary=1)
    assert so["newton_fallbacks"] > 0


def vacuum_state(nodes, tets, ul, ur):
    """rho = 1, p = 0.4 (a = 0.748), u_x = ul left of x = 0.5 and ur right
    of it: across the plane x = 0.5 the normal velocities part by
    ur - ul >= 8 > 2 (a_L + a_R) / (g - 1) = 7.48, so vacuum is generated."""
    c = I.tet_centroids(nodes, tets)
    prim = np.zeros((len(tets), 5))
    prim[:, 0] = 1.0
    prim[:, 4] = 0.4
    prim[:, 1] = np.where(c[:, 0] < 0.5, ul, ur)
    return prim


# (u_L, u_R): the sample at x/t = 0 in the vacuum itself, in the left fan,
# in the right fan
VACUUM = [((-4.0, 4.0), 1, 0), ((-4.0, 4.0), 2, 1), ((-1.0, 7.0), 1, 0), ((-1.0, 7.0), 2, 1),
          ((-7.0, 1.0), 1, 1), ((-7.0, 1.0), 2, 0)]


@pytest.mark.parametrize("vel,order,boundary", VACUUM,
                         ids=[f"u{a:+g}{b:+g}-o{o}-bc{bc}" for (a, b), o, bc in VACUUM])
def test_vacuum_faces(T, orc, vel, order, boundary):
    nodes, tets = I.graded_box_mesh(8, 4, 4, 2.0)
    prim = vacuum_state(nodes, tets, *vel)
    sg, so = run_pair(T, orc, nodes, tets, prim, [1, 2, 7], order, 3, boundary=boundary)
    assert so["vacuum_faces"] > 0


def _mlp_run(T, nodes, tets, prim, guess, theta=None, **kw):
    s = T.Solver(max_levels=5, order=2, guess=guess, guess_stats=1, guess_gate=0.0, **kw)
    s.upload(nodes, tets)
    s.init(prim)
    if theta is not None:
        T.tafv_mlp_set(s.ctx, theta)
    s.advance(8)
    s.advance(8)
    ck, st = s.checkpoint(), s.stats()
    s.close()
    return ck, st


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32flux"])
def test_rejected_network_start_equals_two_rarefaction(T, precision):
    """Zero weights and b3 = +-1000: y = +-1000 on every face, p_TR e^y is
    +inf or 0, and the judge rejects every network start."""
    nodes, tets = I.graded_cube_mesh(16, 16.0)
    prim = I.blast_state(nodes, tets, centre=I.blast_centre(2))
    ck_tr, st_tr = _mlp_run(T, nodes, tets, prim, T.GUESS_TR, precision=precision)
    for b3 in (1000.0, -1000.0):
        th = np.zeros(M.N_PARAMS, np.float32)
        th[-1] = b3
        ck, st = _mlp_run(T, nodes, tets, prim, T.GUESS_MLP, th, precision=precision)
        say(f"b3 {b3:+g}: evaluated {st['guess_evaluated']}, rejected {st['guess_rejected']}, "
            f"used {st['guess_used']}, inexact-TR faces {st['guess_faces']}")
        assert st["guess_rejected"] > 0
        assert st["guess_used"] == 0
        assert st["guess_rejected"] == st["guess_evaluated"] == st["guess_faces"]
        for k in ("cons", "accum", "levels"):
            assert np.array_equal(ck[k], ck_tr[k]), k
        for k in ("cell_updates", "face_solves", "newton_updates", "guess_newton_updates"):
            assert st[k] == st_tr[k], (k, st[k], st_tr[k])


def test_nonfinite_network_parameter(T):
    s = T.Solver(max_levels=3, order=1, guess=T.GUESS_MLP)
    good = M.he_uniform(1).astype(np.float32)
    for bad_value in (np.nan, np.inf, -np.inf):
        th = good.copy()
        th[100] = bad_value
        with pytest.raises(T.TafvError) as e:
            T.tafv_mlp_set(s.ctx, th)
        assert e.value.code == T.E_MLP
    # a refused set leaves no network: advancing with the learned guess fails
    cfg = I.config_small()
    s.upload(cfg["nodes"], cfg["tets"])
    s.init(cfg["prim"])
    with pytest.raises(T.TafvError) as e:
        s.advance(1)
    assert e.value.code == T.E_MLP
    T.tafv_mlp_set(s.ctx, good)
    s.advance(1)
    s.close()


def _oracle_newton_hist(orc, nodes, tets, prim, max_iter=50):
    """Category x update-count histogram of the oracle's Newton solves of
    every face from the cell states (first order, walls), binned as the
    library bins them."""
    mesh = orc.Mesh(nodes, tets)
    g = mesh.geometry()
    w = orc.cons_to_prim(orc.prim_to_cons(prim))
    hist = np.zeros((3, 8), np.int64)
    long_updates = np.zeros(3, np.int64)
    for f in range(mesh.n_faces):
        L, R = int(g["face_L"][f]), int(g["face_R"][f])
        wl = w[L]
        wr = w[R] if R >= 0 else None
        _, out = orc.face_flux(wl, wr, g["face_area"][f],
                               orc.KIND_INTERIOR if R >= 0 else orc.KIND_WALL, max_iter=max_iter)
        if out.vacuum:
            continue
        pl, pr = wl[4], (wr[4] if R >= 0 else wl[4])
        cat = int(out.p_star > min(pl, pr)) + int(out.p_star > max(pl, pr))
        b = min(max(out.newton_updates, 1), 8) - 1
        hist[cat, b] += 1
        if b == 7:
            long_updates[cat] += out.newton_updates
    return hist, long_updates


@pytest.mark.parametrize("max_iter", [50, 2], ids=["newton", "bisection"])
def test_newton_histogram_against_oracle(T, orc, max_iter):
    """Face statistics by category and Newton update count: the first
    subiteration at first order solves every face once from the cell
    states; the library's histogram matches the oracle's solves of the same
    faces, and it sums to the face solves and the Newton updates."""
    nodes, tets = I.graded_box_mesh(10, 8, 6, 4.0)
    prim = I.blast_state(nodes, tets, centre=I.blast_centre(3))
    s = T.Solver(max_levels=4, order=1, guess_stats=1, newton_max_iter=max_iter)
    s.upload(nodes, tets)
    s.init(prim)
    st = s.advance(1)
    s.close()
    h = np.array(st["newton_hist"], np.int64)
    lu = np.array(st["newton_hist_long_updates"], np.int64)
    ho, luo = _oracle_newton_hist(orc, nodes, tets, prim, max_iter)
    say(f"GPU histogram (rows: rarefactions, one shock, two shocks; columns 1..7, 8+ "
        f"updates):\n{h}\noracle:\n{ho}")
    assert h.sum() == st["face_solves"] - st["vacuum_faces"]
    upd = sum((b + 1) * h[:, b].sum() for b in range(7)) + lu.sum()
    assert upd == st["newton_updates"]
    assert h.sum() == ho.sum()
    assert np.abs(h - ho).max() <= 1e-3 * ho.sum() + 5
    assert abs(int(lu.sum()) - int(luo.sum())) <= 1e-3 * max(int(luo.sum()), 1) + 5 * max_iter
    assert h[1:].sum() > 0  # the blast has shocks
    if max_iter == 2:
        assert h[:, 7].sum() == 0 and st["newton_fallbacks"] > 0
