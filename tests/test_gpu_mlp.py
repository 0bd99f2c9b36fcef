"""GPU tests of the learned p* guess: the MFMA network kernels against the
FP64 reference with BF16 emulation (oracle/mlp_ref), GPU training, face
logging, unchanged p* with the learned start, and what the trained network
gains in Newton updates over the two-rarefaction start."""
import sys

import numpy as np
import pytest

from oracle import mlp_ref as M
from paper_1704_01144_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def T():
    from paper_1704_01144_amd import tafv
    return tafv


def shock_faces(orc, n, seed):
    """Random face states (rho, u_n, p) where the two-rarefaction start is
    inexact (at least one shock), with features and targets ln(p*/p_TR)."""
    g = np.random.default_rng(seed)
    wl, wr = [], []
    while len(wl) < n:
        a = np.array([g.uniform(0.3, 3), g.uniform(-1, 1), np.exp(g.uniform(-1.5, 1.5))])
        b = np.array([g.uniform(0.3, 3), g.uniform(-1, 1), np.exp(g.uniform(-1.5, 1.5))])
        rs = orc.riemann_solve(a, b)
        if rs.vacuum or rs.p_star <= min(a[2], b[2]):
            continue
        wl.append(a)
        wr.append(b)
    wl, wr = np.array(wl), np.array(wr)
    x, rm, pm, am = M.features(wl, wr)
    ptr = M.two_rarefaction(wl, wr)
    t = np.array([M.target(orc.riemann_solve(a, b).p_star, p) for a, b, p in zip(wl, wr, ptr)])
    return x, t, wl, wr


def near_bf16_tie(z, mag, rel=4 * 2.0 ** -24):
    """True where a positive pre-activation z lies within rel * mag of a
    midpoint between two BF16 values: there FP32 and FP64 sums (mag the sum
    of the absolute terms; a few FP32 roundings of partial sums bounded by
    it) may round the activation to different BF16 neighbours."""
    z = np.asarray(z, dtype=np.float64)
    pos = z > 0
    e = np.floor(np.log2(np.where(pos, z, 1.0)))
    ulp = 2.0 ** (e - 7)
    frac = np.mod(z / ulp, 1.0)
    dist = np.abs(frac - 0.5) * ulp
    return pos & (dist <= rel * mag)


def test_forward_matches_bf16_emulation(T, orc):
    """Rows whose hidden activations are away from BF16 ties: the GPU
    output equals the BF16-emulating reference to 1e-5 (the FP32 sums of
    the GPU against the FP64 sums of the reference).  The excluded rows are
    counted and must be few."""
    s = T.Solver(max_levels=2, order=1)
    th = M.he_uniform(1) + np.random.default_rng(2).normal(0, 0.05, M.N_PARAMS)
    th32 = th.astype(np.float32)
    T.tafv_mlp_set(s.ctx, th32)
    assert np.array_equal(T.tafv_mlp_get(s.ctx), th32)
    x, t, _, _ = shock_faces(orc, 3000, 3)
    x32 = x.astype(np.float32)
    y = T.tafv_mlp_forward(s.ctx, x32)
    yref, a = M.forward(th32.astype(np.float64), x32.astype(np.float64), emulate_bf16=True)
    p = a["p"]
    mag1 = np.abs(a["x"]) @ np.abs(p["W1"]).T + np.abs(p["b1"])
    mag2 = np.abs(a["h1"]) @ np.abs(p["W2"]).T + np.abs(p["b2"])
    tie = near_bf16_tie(a["z1"], mag1).any(1) | near_bf16_tie(a["z2"], mag2).any(1)
    err = np.abs(y - yref)
    say(f"forward: {int(tie.sum())} of {len(y)} rows near a BF16 tie excluded; others: "
        f"median {np.median(err[~tie]):.2e} max {err[~tie].max():.2e}; all rows max {err.max():.2e}")
    assert tie.sum() <= 0.12 * len(y)
    assert err[~tie].max() <= 1e-5
    s.close()


def test_gradient_matches_reference(T, orc):
    """The training kernels' gradient against the BF16-emulating reference
    backward (BF16 forward activations, dz2 and dz1 rounded to BF16 as the
    operands of the training products): normwise <= 1e-3, and per
    parameter group."""
    s = T.Solver(max_levels=2, order=1)
    th32 = (M.he_uniform(4) + np.random.default_rng(5).normal(0, 0.05, M.N_PARAMS)).astype(np.float32)
    T.tafv_mlp_set(s.ctx, th32)
    x, t, _, _ = shock_faces(orc, 2000, 6)
    x32, t32 = x.astype(np.float32), t.astype(np.float32)
    g, loss = T.tafv_mlp_grad(s.ctx, x32, t32)
    gref = M.backward(th32.astype(np.float64), x32.astype(np.float64), t32.astype(np.float64),
                      emulate_bf16=True)
    lref = M.loss(th32.astype(np.float64), x32.astype(np.float64), t32.astype(np.float64),
                  emulate_bf16=True)
    rel = np.linalg.norm(g - gref) / np.linalg.norm(gref)
    parts = {"W1": (0, 192), "b1": (192, 224), "W2": (224, 1248), "b2": (1248, 1280),
             "w3": (1280, 1312), "b3": (1312, 1313)}
    rg = {k: np.linalg.norm(g[a:b] - gref[a:b]) / max(np.linalg.norm(gref[a:b]), 1e-12)
          for k, (a, b) in parts.items()}
    say(f"gradient: normwise rel err {rel:.2e}, loss {loss:.6f} vs {lref:.6f}; per group " +
        ", ".join(f"{k} {v:.1e}" for k, v in rg.items()))
    assert rel <= 1e-3
    assert abs(loss - lref) < 1e-4 * lref
    for k, v in rg.items():
        assert v <= 3e-3, (k, v)
    s.close()


@pytest.fixture(scope="module")
def trained(T, orc):
    """Train on face states logged by the solver itself: 24^3 hexes graded
    16x, blasts centred by seeds 1-3, 16 dt_min units each."""
    rows = []
    for seed in (1, 2, 3):
        nodes, tets = I.graded_cube_mesh(24, 16.0)
        prim = I.blast_state(nodes, tets, centre=I.blast_centre(seed))
        s = T.Solver(max_levels=5, order=2, guess_stats=1)
        s.upload(nodes, tets)
        s.init(prim)
        T.tafv_facelog_config(s.ctx, 200000, 0.5, seed)
        s.advance(16)
        rows.append(T.tafv_facelog_read(s.ctx, 200000))
        s.close()
    rows = np.concatenate(rows)
    say(f"logged rows: {len(rows)}")
    s = T.Solver(max_levels=2, order=1)
    T.tafv_mlp_set(s.ctx, M.he_uniform(7).astype(np.float32))
    loss = T.tafv_mlp_train(s.ctx, rows[:, :6], rows[:, 6], epochs=30, batch=4096, lr=2e-3,
                            seed=11)
    th = T.tafv_mlp_get(s.ctx)
    s.close()
    say(f"training loss per epoch: first {loss[0]:.3e} last {loss[-1]:.3e}")
    return dict(rows=rows, loss=loss, theta=th)


def _row_states(r):
    """Face states of a logged row: with rho_m = p_m = 1 and u_m = 0 the
    inputs are the states' deviations from (1, 0, 1) (a_m = sqrt(1.4))."""
    x = np.asarray(r[:6], dtype=np.float64)
    am = np.sqrt(1.4)
    return [1.0 + x[0], x[1] * am, 1.0 + x[2]], [1.0 + x[3], x[4] * am, 1.0 + x[5]]


def test_face_log_rows_are_exact(T, orc, trained):
    rows = trained["rows"]
    assert len(rows) > 1000
    sub = rows[np.random.default_rng(8).choice(len(rows), 300, replace=False)]
    for r in sub:
        x = r[:6].astype(np.float64)
        assert abs(x[0] + x[3]) < 1e-7 and abs(x[1] + x[4]) < 1e-7 and abs(x[2] + x[5]) < 1e-7
        wl, wr = _row_states(r)
        rs = orc.riemann_solve(wl, wr)
        ptr = M.two_rarefaction(wl, wr)[0]
        assert ptr > min(wl[2], wr[2]) * (1 - 1e-5)  # the logging gate
        assert abs(np.log(rs.p_star / ptr) - r[6]) < 2e-5 * (1 + abs(r[6]))


def test_face_log_and_training_reproducible(T):
    """Two runs log the same rows in the same order (the rows are sorted by
    their bytes on readback, whichever wave took which slot), and training
    on them twice gives the same network bit for bit."""
    nodes, tets = I.graded_cube_mesh(16, 16.0)
    prim = I.blast_state(nodes, tets, centre=I.blast_centre(2))
    logs, thetas = [], []
    for _ in range(2):
        s = T.Solver(max_levels=5, order=2, guess_stats=1)
        s.upload(nodes, tets)
        s.init(prim)
        T.tafv_facelog_config(s.ctx, 100000, 0.5, 7)
        s.advance(8)
        rows = T.tafv_facelog_read(s.ctx, 100000)
        T.tafv_mlp_set(s.ctx, M.he_uniform(3).astype(np.float32))
        T.tafv_mlp_train(s.ctx, rows[:, :6], rows[:, 6], epochs=3, batch=1024, lr=2e-3, seed=5)
        thetas.append(T.tafv_mlp_get(s.ctx))
        logs.append(rows)
        s.close()
    say(f"reproducible face log: {len(logs[0])} rows")
    assert len(logs[0]) > 100
    assert np.array_equal(logs[0].view(np.uint32), logs[1].view(np.uint32))
    assert np.array_equal(thetas[0].view(np.uint32), thetas[1].view(np.uint32))


def _newton_updates(orc, rows, y, gate):
    """Newton updates on the oracle's solver from p_TR, or from p_TR exp(y)
    where |y| > gate."""
    out = []
    for r, yy in zip(rows, y):
        wl, wr = _row_states(r)
        if abs(yy) > gate:
            ptr = M.two_rarefaction(wl, wr)[0]
            out.append(orc.riemann_solve(wl, wr, guess=ptr * np.exp(float(yy))).newton_updates)
        else:
            out.append(orc.riemann_solve(wl, wr).newton_updates)
    return np.array(out)


def test_training_reduces_loss(trained):
    loss = trained["loss"]
    assert loss[-1] < 0.1 * loss[0]
    assert np.isfinite(loss).all()


def test_learned_start_keeps_pstar(T, orc, trained):
    nodes, tets = I.graded_cube_mesh(24, 16.0)
    prim = I.blast_state(nodes, tets, centre=I.blast_centre(0))
    s = T.Solver(max_levels=5, order=2, guess=T.GUESS_MLP)
    s.upload(nodes, tets)
    s.init(prim)
    T.tafv_mlp_set(s.ctx, trained["theta"])
    s.advance(24)
    ck = s.checkpoint()
    st = s.stats()
    s.close()
    o = orc.State(orc.Mesh(nodes, tets), prim, orc.params(max_levels=5, order=2))
    o.advance(24)
    u_o, _, lev_o = o.read()
    assert (ck["levels"] == lev_o).all()
    scale = np.abs(u_o).max(0)
    err = (np.abs(ck["cons"] - u_o).max(0) / scale).max()
    say(f"learned start: normwise err {err:.2e}, guess faces {st['guess_faces']}, "
        f"rejected {st['guess_rejected']}")
    assert err <= 1e-12
    assert st["guess_faces"] > 0 and st["newton_fallbacks"] == 0


def test_learned_guess_gain(T, orc, trained):
    """Held-out blast (seed 0): Newton updates per face where the
    two-rarefaction start is inexact.  The gate (use the network's correction
    y only where |y| exceeds it) is tuned on training rows with the oracle's
    solver; the gain is then measured on held-out rows (oracle solver) and
    in the GPU solver itself (counters with and without the network).

    What is asserted: the network has learned the correction (its squared
    error on held-out rows is under half the target's variance), and with the
    tuned gate it costs no more than 2% extra Newton updates over the
    two-rarefaction start; whether it saves any is reported, not assumed:
    Newton converges quadratically, so a start saves an update only where it
    beats the two-rarefaction value's own error, which on the weak shocks of
    these blasts is below the BF16 network's resolution."""
    rows = trained["rows"]
    s = T.Solver(max_levels=2, order=1)
    T.tafv_mlp_set(s.ctx, trained["theta"])
    tune = rows[np.random.default_rng(12).choice(len(rows), 1500, replace=False)]
    y_tune = T.tafv_mlp_forward(s.ctx, tune[:, :6])
    s.close()
    base = _newton_updates(orc, tune, y_tune, np.inf).mean()
    cand = [0.0, 1e-3, 3e-3, 1e-2, 3e-2, 1e-1, 3e-1]
    score = [_newton_updates(orc, tune, y_tune, g).mean() for g in cand]
    gate = cand[int(np.argmin(score))]
    say(f"gate tuning on training rows: TR {base:.3f}; " +
        ", ".join(f"{g:g}: {v:.3f}" for g, v in zip(cand, score)) + f" -> gate {gate:g}")
    nodes, tets = I.graded_cube_mesh(24, 16.0)
    prim = I.blast_state(nodes, tets, centre=I.blast_centre(0))
    res = {}
    for guess in (T.GUESS_TR, T.GUESS_MLP):
        s = T.Solver(max_levels=5, order=2, guess=guess, guess_stats=1, guess_gate=gate)
        s.upload(nodes, tets)
        s.init(prim)
        T.tafv_mlp_set(s.ctx, trained["theta"])
        if guess == T.GUESS_TR:
            T.tafv_facelog_config(s.ctx, 50000, 0.2, 99)
        s.advance(24)
        st = s.stats()
        res[guess] = (st["guess_newton_updates"] / max(st["guess_faces"], 1), st["guess_used"])
        if guess == T.GUESS_TR:
            held = T.tafv_facelog_read(s.ctx, 50000)[:2000]
            y = T.tafv_mlp_forward(s.ctx, held[:, :6])
        s.close()
    m_tr = _newton_updates(orc, held, y, np.inf).mean()
    m_mlp = _newton_updates(orc, held, y, gate).mean()
    mse = float(np.mean((y - held[:, 6]) ** 2))
    var = float(np.var(held[:, 6]))
    strong = np.abs(held[:, 6]) > 0.02  # faces where two-rarefaction is off by > 2%
    if strong.any():
        s_tr = _newton_updates(orc, held[strong], y[strong], np.inf).mean()
        s_nn = _newton_updates(orc, held[strong], y[strong], 0.0).mean()
        say(f"held-out faces with |ln(p*/p_TR)| > 0.02: {int(strong.sum())}, Newton updates "
            f"TR {s_tr:.3f} -> network {s_nn:.3f}")
    say(f"held-out shock faces: network MSE {mse:.2e} vs target variance {var:.2e}; oracle "
        f"solver: TR {m_tr:.3f} -> network {m_mlp:.3f} Newton updates per face; GPU solver: "
        f"TR {res[T.GUESS_TR][0]:.3f} -> network {res[T.GUESS_MLP][0]:.3f} (network start on "
        f"{res[T.GUESS_MLP][1]} faces)")
    assert mse < 0.5 * var
    assert min(score) <= 1.02 * base
    assert m_mlp <= 1.02 * m_tr
    assert res[T.GUESS_MLP][0] <= 1.02 * res[T.GUESS_TR][0]
