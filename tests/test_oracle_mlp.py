"""Pins of the oracle's reference of the p* network:
  * backward against central finite differences (FP64);
  * BF16 rounding against torch's own float32 -> bfloat16 conversion;
  * the input normalisation against the scaling symmetry of the Euler
    equations: scaled face states give the same features and the same
    target ln(p*/p_m) from the (separately pinned) exact Riemann solver;
  * a hand-built network whose output has a closed form.
"""
import numpy as np
import pytest

from oracle import mlp_ref as M


def test_param_count():
    assert M.N_PARAMS == 1313
    th = M.he_uniform(0)
    assert np.array_equal(M.pack(M.unpack(th)), th)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    th = M.he_uniform(2) + rng.normal(0, 0.05, M.N_PARAMS)
    x = rng.normal(0, 1, (64, 6))
    t = rng.normal(0, 0.3, 64)
    g = M.backward(th, x, t)
    h = 1e-6
    idx = rng.choice(M.N_PARAMS, 200, replace=False)
    for k in idx:
        e = np.zeros(M.N_PARAMS)
        e[k] = h
        fd = (M.loss(th + e, x, t) - M.loss(th - e, x, t)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd)), (k, fd, g[k])


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    v = np.concatenate([rng.normal(0, 1, 5000), rng.normal(0, 1e-3, 2000) * 1e3,
                        [1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 0.0, 65504.0, 1e-30]])
    ref = torch.tensor(v.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.bf16(v), ref)


def test_features_follow_scaling_symmetry(orc):
    """Scaling rho -> s rho, u -> c u + v, p -> s c^2 p (a shift v of the
    velocity: Galilean invariance of the star pressure) leaves the features
    and the target unchanged."""
    rng = np.random.default_rng(4)
    for _ in range(200):
        wl = np.array([rng.uniform(0.2, 5), rng.uniform(-1, 1), rng.uniform(0.1, 10)])
        wr = np.array([rng.uniform(0.2, 5), rng.uniform(-1, 1), rng.uniform(0.1, 10)])
        s, c, v = rng.uniform(0.1, 10), rng.uniform(0.1, 10), rng.uniform(-3, 3)
        sl = np.array([s * wl[0], c * wl[1] + v, s * c * c * wl[2]])
        sr = np.array([s * wr[0], c * wr[1] + v, s * c * c * wr[2]])
        x1, _, pm1, _ = M.features(wl, wr)
        x2, _, pm2, _ = M.features(sl, sr)
        assert np.abs(x1 - x2).max() < 1e-13
        r1 = orc.riemann_solve(wl, wr)
        r2 = orc.riemann_solve(sl, sr)
        if r1.vacuum:
            continue
        t1 = M.target(r1.p_star, M.two_rarefaction(wl, wr)[0])
        t2 = M.target(r2.p_star, M.two_rarefaction(sl, sr)[0])
        assert abs(t1 - t2) < 1e-11


def test_two_rarefaction_value(orc):
    """Exact when both waves are rarefactions (target 0); with a shock it is a
    positive estimate whose error grows with the shock strength."""
    rng = np.random.default_rng(9)
    n_rare = 0
    for _ in range(2000):
        wl = np.array([rng.uniform(0.2, 5), rng.uniform(-1, 1), rng.uniform(0.1, 10)])
        wr = np.array([rng.uniform(0.2, 5), rng.uniform(-1, 1), rng.uniform(0.1, 10)])
        rs = orc.riemann_solve(wl, wr)
        if rs.vacuum:
            continue
        ptr = M.two_rarefaction(wl, wr)[0]
        if rs.p_star <= min(wl[2], wr[2]):
            assert abs(ptr - rs.p_star) < 1e-13 * rs.p_star
            n_rare += 1
        else:
            assert np.isfinite(ptr) and ptr > 0
    assert n_rare > 100
    # a strong shock (100:1 at rest) is far from the two-rarefaction value
    rs = orc.riemann_solve([1.0, 0.0, 100.0], [1.0, 0.0, 1.0])
    ptr = M.two_rarefaction([1.0, 0.0, 100.0], [1.0, 0.0, 1.0])[0]
    assert abs(np.log(rs.p_star / ptr)) > 1e-2


def test_hand_built_network():
    # h1_j = relu(x_j) for j < 6 (identity rows), h2 = h1, y = sum of the
    # first three hidden units minus the fourth plus 0.5:
    # y = relu(x0) + relu(x1) + relu(x2) - relu(x3) + 0.5
    p = {"W1": np.zeros((32, 6)), "b1": np.zeros(32), "W2": np.zeros((32, 32)),
         "b2": np.zeros(32), "w3": np.zeros(32), "b3": 0.5}
    p["W1"][:6, :6] = np.eye(6)
    p["W2"][:6, :6] = np.eye(6)
    p["w3"][:4] = [1, 1, 1, -1]
    th = M.pack(p)
    x = np.random.default_rng(5).normal(0, 1, (100, 6))
    y, _ = M.forward(th, x)
    r = np.maximum(x, 0)
    assert np.allclose(y, r[:, 0] + r[:, 1] + r[:, 2] - r[:, 3] + 0.5, rtol=0, atol=1e-15)
    # BF16 emulation of the same network is exact for BF16-representable inputs
    xb = M.bf16(x)
    yb, _ = M.forward(th, xb, emulate_bf16=True)
    rb = np.maximum(xb, 0)
    assert np.allclose(yb, rb[:, 0] + rb[:, 1] + rb[:, 2] - rb[:, 3] + 0.5, rtol=0, atol=1e-15)
