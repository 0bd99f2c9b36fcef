"""Pins of the oracle's reference of the p* network:
  * backward against central finite differences (FP64);
  * BF16 rounding against torch's own float32 -> bfloat16 conversion;
  * the input normalisation against the scaling symmetry of the Euler
    equations: scaled face states give the same features and the same
    target ln(p*/p_m) from the (separately pinned) exact Riemann solver;
  * a hand-built network whose output has a closed form;
  * the BF16 emulation of the backward pass: two single-path networks whose
    emulated gradients have closed forms (dz2 and dz1 rounded to BF16, dy
    not), and a network whose intermediates are all BF16 values, where the
    emulated gradient equals the FP64 one bit for bit.
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


def _single_path(dy, w2, x0=1.0):
    """One row through hidden unit 0 of both layers: x0 -> h1_0 = x0 ->
    h2_0 = w2 x0 -> y = h2_0 (w3_0 = 1, everything else 0), with the target
    set so that dy = 2 (y - t) takes the given value."""
    p = {"W1": np.zeros((32, 6)), "b1": np.zeros(32), "W2": np.zeros((32, 32)),
         "b2": np.zeros(32), "w3": np.zeros(32), "b3": 0.0}
    p["W1"][0, 0] = 1.0
    p["W2"][0, 0] = w2
    p["w3"][0] = 1.0
    x = np.zeros((1, 6))
    x[0, 0] = x0
    y = w2 * x0
    t = np.array([y - dy / 2.0])
    return M.pack(p), x, t


def test_bf16_backward_rounds_dz2_closed_form():
    """dy = 1 + 2^-10 is not a BF16 value: the emulated backward rounds
    dz2 = dy w3 to 1 (the spacing of BF16 at 1 is 2^-7), so the gradients
    of W2, b2, W1 and b1 see 1, while w3 and b3 see dy itself."""
    dy = 1.0 + 2.0 ** -10
    th, x, t = _single_path(dy, 1.0)
    g64 = M.unpack(M.backward(th, x, t))
    g16 = M.unpack(M.backward(th, x, t, emulate_bf16=True))
    assert g64["W2"][0, 0] == dy and g16["W2"][0, 0] == 1.0
    assert g64["b2"][0] == dy and g16["b2"][0] == 1.0
    assert g64["W1"][0, 0] == dy and g16["W1"][0, 0] == 1.0
    assert g64["b1"][0] == dy and g16["b1"][0] == 1.0
    assert g64["w3"][0] == dy and g16["w3"][0] == dy
    assert g64["b3"] == dy and g16["b3"] == dy


def test_bf16_backward_rounds_dz1_closed_form():
    """dz2 = dy = 1.5 is a BF16 value, W2 = 1 + 2^-7 too, but their product
    1.51171875 (binary 1.10000011) is not: it ties between 1.1000001 and
    1.1000010 and rounds to the even one, 1.515625.  That is dz1, and the
    gradients of W1 and b1 (x0 = 1) under emulation."""
    th, x, t = _single_path(1.5, 1.0 + 2.0 ** -7)
    g64 = M.unpack(M.backward(th, x, t))
    g16 = M.unpack(M.backward(th, x, t, emulate_bf16=True))
    assert g64["W1"][0, 0] == 1.51171875 and g16["W1"][0, 0] == 1.515625
    assert g64["b1"][0] == 1.51171875 and g16["b1"][0] == 1.515625
    # dz2 is exact, so the second layer's gradient is the same in both
    assert g64["W2"][0, 0] == g16["W2"][0, 0] == 1.5


def _sparse_dyadic_network(rng):
    """Parameters with at most two non-zeros per row and column of each
    layer, all small dyadic values, so every forward and backward
    intermediate of eight rows of dyadic inputs is a short dyadic number."""
    p = {"W1": np.zeros((32, 6)), "b1": np.zeros(32), "W2": np.zeros((32, 32)),
         "b2": np.zeros(32), "w3": np.zeros(32), "b3": 0.25}
    vals = np.array([-1.0, -0.5, 0.5, 1.0])
    for j in range(32):
        p["W1"][j, j % 6] = rng.choice(vals)
        p["W2"][j, j] = rng.choice(vals)
        p["W2"][j, (j + 1) % 32] = rng.choice(vals)
    p["b1"] = rng.choice([0.0, 0.25, -0.25], 32)
    p["b2"] = rng.choice([0.0, 0.125, 0.5], 32)
    p["w3"] = rng.choice([-1.0, -0.5, -0.25, 0.25, 0.5, 1.0], 32)
    x = rng.choice([-1.375, -0.59375, 0.0, 0.8125, 1.1875, 1.5], (8, 6))
    return M.pack(p), x


def test_bf16_backward_exact_when_values_are_bf16():
    """When every intermediate is a BF16 value, the rounding in the
    emulated forward and backward changes nothing: the emulated gradient
    equals the FP64 gradient bit for bit.  The gradients themselves (sums
    over rows) are not all BF16 values, so rounding a sum would show."""
    rng = np.random.default_rng(21)
    th, x = _sparse_dyadic_network(rng)
    y, a = M.forward(th, x)
    for key in ("x", "z1", "h1", "z2", "h2"):
        assert np.array_equal(M.bf16(a[key]), a[key]), key
    t = y - rng.choice([-1.0, -0.5, 0.5, 1.0], len(y))  # y - t is a short dyadic
    g64 = M.backward(th, x, t)
    g16 = M.backward(th, x, t, emulate_bf16=True)
    assert np.array_equal(g64, g16)
    assert (M.bf16(g64) != g64).sum() >= 5
    assert np.count_nonzero(g64) > 100
