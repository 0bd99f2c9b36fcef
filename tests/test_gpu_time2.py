"""GPU parity of the predictor/corrector form of the level steps
(time_order = 2; Sec. 2.2, Alg. 2: predictor, prediction, interpolation of
the slower levels, corrector, correction) against the oracle's form.

Bar (FP64): per conserved component k,
  max_i |U_ik(gpu) - U_ik(oracle)| / max_i |U_ik(oracle)| <= 1e-12,
identical levels and schedule counters; FP32 flux: L1 error of density and
energy <= 1e-5 against the FP64 oracle.  Also: conservation at every
subiteration on the device state, second-order convergence in time measured
on the device, reset and checkpoint rules, and the full benchmark mesh
(1,572,864 cells, 32 units) cell by cell.
"""
import sys

import numpy as np
import pytest

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
    scale = np.abs(b).max(0)
    scale[scale == 0] = 1.0
    return (np.abs(a - b).max(0) / scale).max()


def l1_rel(a, b, vol):
    return (vol * np.abs(a - b)).sum() / (vol * np.abs(b)).sum()


def run_pair(T, orc, nodes, tets, prim, order, L, chunks, precision=0, boundary=0,
             reclassify=1):
    say(f"case: time order 2, cells={len(tets)} order={order} L={L} chunks={chunks} "
        f"precision={precision} boundary={boundary}")
    s = T.Solver(max_levels=L, order=order, precision=precision, boundary=boundary,
                 reclassify=reclassify, time_order=2)
    s.upload(nodes, tets)
    s.init(prim)
    m = orc.Mesh(nodes, tets)
    o = orc.State(m, prim, orc.params(max_levels=L, order=order, boundary=boundary,
                                      reclassify=reclassify, time_order=2))
    for n in chunks:
        s.advance(n)
        o.advance(n)
        ck = s.checkpoint()
        u_o, r_o, lev_o = o.read()
        assert (ck["levels"] == lev_o).all()
        if precision == 0:
            err = normwise(ck["cons"], u_o)
            scale = np.abs(r_o).max(0)
            scale[scale == 0] = 1.0
            err_r = (np.abs(ck["accum"] - r_o).max(0) / scale).max()
            say(f"  after {n}: normwise err {err:.3e}, accumulators {err_r:.3e}")
            assert err <= TOL and err_r <= 1e-11, (err, err_r)
    sg, so = s.stats(), o.stats()
    for k in ("subiterations", "cell_updates", "face_solves", "theta", "phase"):
        assert sg[k] == so[k], (k, sg[k], so[k])
    assert sg["cells_per_level"] == so["cells_per_level"]
    assert abs(sg["newton_updates"] - so["newton_updates"]) <= 1e-3 * so["newton_updates"] + 5
    imp_g, imp_o = np.array(sg["wall_impulse"]), np.array(so["wall_impulse"])
    assert np.abs(imp_g - imp_o).max() <= 1e-12 * max(np.abs(imp_o).max(), 1e-300) + 1e-15
    u_g = s.checkpoint()["cons"]
    s.close()
    return u_g, o, m, sg


def test_small_first_order(T, orc):
    cfg = I.config_small()
    u, o, m, st = run_pair(T, orc, cfg["nodes"], cfg["tets"], cfg["prim"], 1, 3,
                           [1, 1, 1, 1, 2, 2])
    assert st["theta"] == 2


def test_graded_24_second_order(T, orc):
    nodes, tets = I.graded_cube_mesh(24, 16.0)
    prim = I.blast_state(nodes, tets, centre=I.blast_centre(0))
    u, o, m, st = run_pair(T, orc, nodes, tets, prim, 2, 5, [3, 5, 8, 16])
    assert st["theta"] >= 2


def test_ragged_and_tiny_meshes(T, orc):
    for xs, ys, zs, L, order in [([0, 1], [0, 1], [0, 1], 2, 2),
                                 (I.graded_coords(5, 3.0), I.graded_coords(7, 2.0),
                                  I.graded_coords(3, 1.0), 4, 2),
                                 (I.graded_coords(9, 5.0), I.graded_coords(4, 1.0),
                                  I.graded_coords(6, 2.0), 1, 1)]:
        nodes, tets = I.kuhn_tet_mesh(np.array(xs, float), np.array(ys, float),
                                      np.array(zs, float))
        prim = I.random_state(len(tets), 11)
        run_pair(T, orc, nodes, tets, prim, order, L, [5, 7])


def test_transmissive_and_fixed_levels(T, orc):
    nodes, tets = I.graded_box_mesh(10, 8, 6, 8.0)
    prim = I.pulse_state(nodes, tets, amp=0.2, velocity=(0.3, -0.1, 0.2))
    run_pair(T, orc, nodes, tets, prim, 2, 4, [4, 9, 3], boundary=T.BC_TRANSMIT, reclassify=0)


def test_fp32_form_l1(T, orc):
    nodes, tets = I.graded_cube_mesh(24, 16.0)
    prim = I.blast_state(nodes, tets, centre=I.blast_centre(0))
    s = T.Solver(max_levels=5, order=2, precision=T.FP32_FLUX, time_order=2)
    s.upload(nodes, tets)
    s.init(prim)
    s.advance(32)
    ck = s.checkpoint()
    s.close()
    m = orc.Mesh(nodes, tets)
    o = orc.State(m, prim, orc.params(max_levels=5, order=2, time_order=2))
    o.advance(32)
    u_o, _, lev_o = o.read()
    vol = m.geometry()["vol"]
    e_rho = l1_rel(ck["cons"][:, 0], u_o[:, 0], vol)
    e_E = l1_rel(ck["cons"][:, 4], u_o[:, 4], vol)
    say(f"time order 2, fp32 form: L1 rho {e_rho:.3e}  L1 E {e_E:.3e}")
    assert e_rho <= 1e-5 and e_E <= 1e-5


def test_conservation_every_subiteration(T, orc):
    nodes, tets = I.graded_cube_mesh(12, 8.0)
    prim = I.blast_state(nodes, tets, centre=(0.3, 0.6, 0.45))
    prim[:, 1:4] = np.random.default_rng(3).uniform(-0.3, 0.3, (len(tets), 3))
    vol = orc.Mesh(nodes, tets).geometry()["vol"][:, None]
    for precision in (0, 1):
        s = T.Solver(max_levels=4, order=2, precision=precision, time_order=2)
        s.upload(nodes, tets)
        s.init(prim)
        tot0 = (vol * orc.prim_to_cons(prim)).sum(0)
        for k in range(16):
            s.advance(1)
            ck = s.checkpoint()
            tot = (vol * ck["cons"]).sum(0) + ck["accum"].sum(0)
            for c in (0, 4):
                assert abs(tot[c] - tot0[c]) < 1e-13 * abs(tot0[c]), (precision, k, c)
            st = s.stats()
            mom = tot[1:4] + np.array(st["wall_impulse"])
            scale = (vol * np.abs(ck["cons"][:, 1:4])).sum() + (vol * ck["cons"][:, :1]).sum()
            assert np.abs(mom - tot0[1:4]).max() < 1e-13 * scale
        assert st["theta"] >= 2
        s.close()


def test_second_order_in_time_on_device(T, orc):
    """Error at a fixed final time against a fine global-step run falls by
    about 4 per halving of the time steps, across four levels."""
    nodes, tets = I.graded_box_mesh(6, 6, 6, 16.0)
    prim = I.pulse_state(nodes, tets)

    def run(cfl, L, units):
        s = T.Solver(max_levels=L, order=2, reclassify=0, time_order=2, cfl=cfl)
        s.upload(nodes, tets)
        s.init(prim)
        st = s.advance(units)
        u = s.read()[0]
        s.close()
        return u, st

    _, st = run(0.4, 4, 1)
    theta = st["theta"]
    assert theta == 3
    units = 2 * 2 ** theta
    u_ref, st_ref = run(0.4 / 32, 1, 32 * units)
    errs = []
    for k in (1, 2, 4):
        u, st = run(0.4 / k, 4, k * units)
        assert abs(st["t_reached"] - st_ref["t_reached"]) <= 1e-12 * st_ref["t_reached"]
        errs.append(np.abs(u - u_ref).max())
    say(f"time order 2 on the device: errors {errs}")
    assert min(errs[0] / errs[1], errs[1] / errs[2]) > 3.6


def test_reset_checkpoint_and_errors(T):
    nodes, tets = I.graded_cube_mesh(10, 8.0)
    prim = I.blast_state(nodes, tets, centre=I.blast_centre(3))
    s = T.Solver(max_levels=4, order=2, time_order=2)
    s.upload(nodes, tets)
    s.init(prim)
    s.advance(7)
    a = s.checkpoint()
    assert a["phase"] != 0
    with pytest.raises(T.TafvError) as e:
        s.restore(a)
    assert e.value.code == T.E_ARG
    s.reset()
    s.advance(7)
    b = s.checkpoint()
    assert np.array_equal(a["cons"], b["cons"]) and np.array_equal(a["accum"], b["accum"])
    # a phase-0 checkpoint restores into a fresh context and continues bitwise
    s.advance(2 ** b["theta"] - b["phase"])
    c0 = s.checkpoint()
    assert c0["phase"] == 0
    s.advance(5)
    c1 = s.checkpoint()
    s.close()
    s = T.Solver(max_levels=4, order=2, time_order=2)
    s.upload(nodes, tets)
    s.init(prim)
    s.restore(c0)
    s.advance(5)
    assert np.array_equal(s.checkpoint()["cons"], c1["cons"])
    s.close()
    for kw in (dict(time_order=3), dict(time_order=2, scatter=T.SCATTER_COLOUR),
               dict(time_order=2, batch=1)):
        with pytest.raises(T.TafvError) as e:
            T.Solver(**kw)
        assert e.value.code == T.E_ARG


@pytest.fixture(scope="module")
def full_oracle2(orc):
    """The benchmark workload advanced by the oracle's predictor/corrector
    form: 64^3 hexes graded 16x (1,572,864 cells), second order, L = 5,
    32 dt_min units from t = 0."""
    cfg = I.config_scale(64, 0)
    m = orc.Mesh(cfg["nodes"], cfg["tets"])
    o = orc.State(m, cfg["prim"], orc.params(max_levels=5, order=2, time_order=2))
    say("oracle (time order 2): 32 units on the full mesh ...")
    o.advance(32)
    u_o, _, lev_o = o.read()
    return dict(cfg=cfg, cons=u_o, levels=lev_o, stats=o.stats())


@pytest.mark.parametrize("cell_order", [1, 0], ids=["morton", "mesh-order"])
def test_full_scale_whole_run(T, full_oracle2, cell_order):
    """The benchmark step in the predictor/corrector form, every cell, with
    the cells in Morton order inside the library (the benchmark's
    configuration) and in the mesh's own order."""
    cfg = full_oracle2["cfg"]
    s = T.Solver(max_levels=5, order=2, time_order=2, cell_order=cell_order)
    s.upload(cfg["nodes"], cfg["tets"])
    s.init(cfg["prim"])
    st = s.advance(32)
    cons, lev = s.read()
    s.close()
    err = normwise(cons, full_oracle2["cons"])
    say(f"full run, time order 2, cell order {cell_order}: err {err:.2e}, updates "
        f"{st['cell_updates']}, face solves {st['face_solves']}")
    assert err <= TOL
    assert (lev == full_oracle2["levels"]).all()
    assert st["cell_updates"] == full_oracle2["stats"]["cell_updates"]
    assert st["face_solves"] == full_oracle2["stats"]["face_solves"]


def test_learned_start_same_result(T):
    """The learned start changes only where the Newton iteration begins; the
    predictor/corrector result equals the two-rarefaction start's."""
    from oracle import mlp_ref as M
    nodes, tets = I.graded_cube_mesh(16, 16.0)
    prim = I.blast_state(nodes, tets, centre=I.blast_centre(4))
    th = (M.he_uniform(7) + np.random.default_rng(8).normal(0, 0.05, M.N_PARAMS)).astype(np.float32)
    out = []
    for guess in (T.GUESS_TR, T.GUESS_MLP):
        s = T.Solver(max_levels=5, order=2, time_order=2, guess=guess, guess_stats=1)
        s.upload(nodes, tets)
        if guess == T.GUESS_MLP:
            T.tafv_mlp_set(s.ctx, th)
        s.init(prim)
        st = s.advance(16)
        out.append((s.checkpoint(), st))
        s.close()
    (a, sa), (b, sb) = out
    err = normwise(b["cons"], a["cons"])
    say(f"time order 2, learned start: err {err:.2e}, network start on {sb['guess_used']} of "
        f"{sb['guess_faces']} faces")
    assert err <= TOL and (a["levels"] == b["levels"]).all()
    assert sb["guess_used"] > 0 and sb["newton_fallbacks"] == 0
    assert sa["face_solves"] == sb["face_solves"]
