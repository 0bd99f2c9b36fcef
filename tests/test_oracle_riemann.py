"""Pins of the oracle's exact Riemann solver and Godunov face flux
(Sec. 2.1: fluxes from a Riemann problem per face, Godunov's method).

Every check here is independent of the solver's own pressure functions:
  * brute force: p* from bisection on a pressure function derived anew in
    this file from the Hugoniot curve and the Rankine-Hugoniot mass flux
    (shocks) and from isentropy plus the Riemann invariant (rarefactions);
  * closed forms: identical states, symmetric rarefaction, symmetric
    collision (a quadratic), two-rarefaction data where that guess is exact;
  * invariants of the sampled solution: Rankine-Hugoniot jump conditions with
    the shock speed from the mass equation, Riemann invariants and entropy
    through fans, continuity of p and u across the contact;
  * flux consistency F(W, W) = F(W), rotation equivariance, antisymmetry.
"""
import numpy as np
import pytest

G = 1.4


def sound(rho, p):
    return np.sqrt(G * p / rho)


def f_side_independent(p, rho, pk):
    """Velocity change across the wave of one side, from first principles:
    shock: Hugoniot density ratio + mass flux Q^2 = (p - pk)/(1/rho - 1/rho*);
    rarefaction: rho* = rho (p/pk)^(1/G) and u + 2a/(G-1) invariant."""
    p = np.asarray(p, dtype=np.float64)
    shock = p > pk
    rs = rho * ((G + 1) * p + (G - 1) * pk) / ((G - 1) * p + (G + 1) * pk)
    with np.errstate(divide="ignore", invalid="ignore"):
        Q = np.sqrt((p - pk) / (1.0 / rho - 1.0 / rs))
        f_sh = (p - pk) / Q
    rr = rho * (p / pk) ** (1.0 / G)
    f_ra = 2.0 / (G - 1) * (np.sqrt(G * p / rr) - sound(rho, pk))
    return np.where(shock, f_sh, f_ra)


def pstar_bisection(wl, wr, iters=300):
    """wl, wr: arrays [n][3] of (rho, u, p).  Vectorised bisection."""
    def F(p):
        return (f_side_independent(p, wl[:, 0], wl[:, 2]) +
                f_side_independent(p, wr[:, 0], wr[:, 2]) + wr[:, 1] - wl[:, 1])
    lo = np.zeros(len(wl))
    hi = np.maximum(wl[:, 2], wr[:, 2])
    for _ in range(200):
        grow = F(hi) <= 0
        if not grow.any():
            break
        hi = np.where(grow, 2 * hi, hi)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        pos = F(mid) > 0
        hi = np.where(pos, mid, hi)
        lo = np.where(pos, lo, mid)
    return 0.5 * (lo + hi)


def random_faces(n, seed, strong=True):
    g = np.random.default_rng(seed)
    wl = np.stack([np.exp(g.uniform(np.log(0.1), np.log(10), n)), g.uniform(-2, 2, n),
                   np.exp(g.uniform(np.log(0.01), np.log(100), n))], 1)
    wr = np.stack([np.exp(g.uniform(np.log(0.1), np.log(10), n)), g.uniform(-2, 2, n),
                   np.exp(g.uniform(np.log(0.01), np.log(100), n))], 1)
    if not strong:
        wr = wl * (1 + g.uniform(-0.01, 0.01, (n, 3)))
    # drop data that generate vacuum
    ok = 2 * (sound(wl[:, 0], wl[:, 2]) + sound(wr[:, 0], wr[:, 2])) / (G - 1) > wr[:, 1] - wl[:, 1]
    return wl[ok], wr[ok]


def test_pstar_matches_independent_bisection(orc):
    wl, wr = random_faces(10000, 1)
    # blast-like 10:1 pressure jumps at rest
    wl = np.concatenate([wl, [[1.0, 0.0, 10.0], [1.0, 0.0, 1.0]]])
    wr = np.concatenate([wr, [[1.0, 0.0, 1.0], [1.0, 0.0, 10.0]]])
    ref = pstar_bisection(wl, wr)
    got = np.array([orc.riemann_solve(a, b).p_star for a, b in zip(wl, wr)])
    rel = np.abs(got - ref) / ref
    assert rel.max() < 1e-12, rel.max()
    outs = [orc.riemann_solve(a, b) for a, b in zip(wl, wr)]
    assert not any(o.fallback for o in outs)  # Newton converged everywhere
    assert np.mean([o.newton_updates for o in outs]) < 5


def test_guess_changes_only_iterations(orc):
    wl, wr = random_faces(2000, 2)
    g = np.random.default_rng(3)
    for a, b in zip(wl, wr):
        ref = orc.riemann_solve(a, b)
        for guess in (g.uniform(1e-3, 1e3), ref.p_star * (1 + 1e-3), 1e-6):
            out = orc.riemann_solve(a, b, guess=guess)
            assert abs(out.p_star - ref.p_star) <= 1e-13 * ref.p_star + 1e-300
            assert out.fallback == 0
    # a rejected guess (non-positive, non-finite) falls back to the TR guess
    a, b = wl[0], wr[0]
    ref = orc.riemann_solve(a, b)
    for bad in (-1.0, 0.0, np.nan, np.inf):
        out = orc.riemann_solve(a, b, guess=bad)
        assert out.p_star == ref.p_star and out.newton_updates == ref.newton_updates


def test_closed_forms(orc):
    # identical states: p* = p, u* = u
    for w in ([1.0, 0.3, 2.0], [0.2, -1.5, 0.05], [5.0, 0.0, 100.0]):
        out = orc.riemann_solve(w, w)
        assert abs(out.p_star - w[2]) < 1e-14 * w[2]
        assert abs(out.u_star - w[1]) < 1e-14 * max(1, abs(w[1]))
    # symmetric rarefaction (-U | +U)
    rho, p, U = 1.3, 2.0, 0.7
    a = sound(rho, p)
    exact = p * (1 - (G - 1) * U / (2 * a)) ** (2 * G / (G - 1))
    out = orc.riemann_solve([rho, -U, p], [rho, U, p])
    assert abs(out.p_star - exact) < 1e-14 * exact and abs(out.u_star) < 1e-15
    # TR is exact for two rarefactions -> the first update already stops
    assert out.newton_updates == 1
    # symmetric collision (+U | -U): two shocks, A (p - p0)^2 = U^2 (p + B)
    A, B = 2 / ((G + 1) * rho), (G - 1) / (G + 1) * p
    b = -(2 * A * p + U * U)
    c = A * p * p - U * U * B
    exact = (-b + np.sqrt(b * b - 4 * A * c)) / (2 * A)
    out = orc.riemann_solve([rho, U, p], [rho, -U, p])
    assert abs(out.p_star - exact) < 1e-13 * exact and abs(out.u_star) < 1e-15


def test_wall_flux_closed_forms(orc):
    area = np.array([0.0, 0.0, 0.5])  # |A| = 0.5, n = +z
    rho, p = 0.8, 1.5
    a = sound(rho, p)
    for un in (-0.6, 0.0, 0.9):
        w = np.array([rho, 0.2, -0.1, un, p])
        flux, out = orc.face_flux(w, None, area, kind=orc.KIND_WALL)
        if un < 0:
            pstar = p * (1 + (G - 1) * un / (2 * a)) ** (2 * G / (G - 1))
        else:
            A, B = 2 / ((G + 1) * rho), (G - 1) / (G + 1) * p
            bq = -(2 * A * p + un * un)
            cq = A * p * p - un * un * B
            pstar = (-bq + np.sqrt(bq * bq - 4 * A * cq)) / (2 * A)
        assert flux[0] == 0.0 and flux[4] == 0.0
        assert abs(flux[3] - 0.5 * pstar) < 1e-13 * pstar
        assert flux[1] == 0.0 and flux[2] == 0.0


def _cons1d(w):
    rho, u, p = w
    return np.array([rho, rho * u, p / (G - 1) + 0.5 * rho * u * u])


def _flux1d(w):
    rho, u, p = w
    E = p / (G - 1) + 0.5 * rho * u * u
    return np.array([rho * u, rho * u * u + p, u * (E + p)])


def test_shock_jump_conditions(orc):
    wl, wr = random_faces(3000, 4)
    n_checked = 0
    for a, b in zip(wl, wr):
        rs = orc.riemann_solve(a, b)
        for side, w in ((0, a), (1, b)):
            if rs.p_star <= w[2] * (1 + 1e-6):
                continue
            # star state just on this side of the contact
            eps = 1e-9 * (abs(rs.u_star) + sound(w[0], w[2]))
            xi = rs.u_star - eps if side == 0 else rs.u_star + eps
            ws, s = orc.riemann_sample(a, b, rs, xi)
            if ws[2] != rs.p_star:
                continue  # xi fell outside the star region (very weak shock)
            Us, Uk = _cons1d(ws), _cons1d(w)
            S = (Us[1] - Uk[1]) / (Us[0] - Uk[0])  # shock speed from mass
            jump = _flux1d(ws) - _flux1d(w) - S * (Us - Uk)
            scale = np.abs(_flux1d(ws)).max() + abs(S) * np.abs(Us).max()
            assert np.abs(jump).max() < 1e-11 * scale
            # the sampler puts the shock at that speed
            d = 1e-7 * (abs(S) + 1)
            w_out, _ = orc.riemann_sample(a, b, rs, S - d if side == 0 else S + d)
            w_in, _ = orc.riemann_sample(a, b, rs, S + d if side == 0 else S - d)
            assert np.allclose(w_out, w, rtol=1e-14)
            assert abs(w_in[2] - rs.p_star) < 1e-12 * rs.p_star
            n_checked += 1
    assert n_checked > 1000


def test_rarefaction_invariants_and_contact(orc):
    wl, wr = random_faces(2000, 5)
    n_fans = 0
    for a, b in zip(wl, wr):
        rs = orc.riemann_solve(a, b)
        # continuity of p and u across the contact
        e = 1e-10 * (1 + abs(rs.u_star))
        w1, s1 = orc.riemann_sample(a, b, rs, rs.u_star - e)
        w2, s2 = orc.riemann_sample(a, b, rs, rs.u_star + e)
        assert s1 == 0 and s2 == 1
        assert abs(w1[2] - w2[2]) <= 1e-14 * w1[2] and abs(w1[1] - w2[1]) <= 1e-13 * (1 + abs(w1[1]))
        if rs.p_star < a[2]:
            al = sound(a[0], a[2])
            head = a[1] - al
            tail = rs.u_star - sound(a[0] * (rs.p_star / a[2]) ** (1 / G), rs.p_star)
            for xi in np.linspace(head, tail, 7)[1:-1]:
                w, _ = orc.riemann_sample(a, b, rs, xi)
                aw = sound(w[0], w[2])
                assert abs(w[1] + 2 * aw / (G - 1) - (a[1] + 2 * al / (G - 1))) < 1e-12 * (1 + al)
                assert abs(w[2] / w[0] ** G - a[2] / a[0] ** G) < 1e-12 * a[2] / a[0] ** G
                assert abs(w[1] - aw - xi) < 1e-12 * (1 + abs(xi))  # left characteristic
            # fan edges meet the outer and star states (tie invariance)
            wh, _ = orc.riemann_sample(a, b, rs, head + 1e-12)
            assert np.allclose(wh, a, rtol=1e-9)
            wt, _ = orc.riemann_sample(a, b, rs, tail - 1e-12)
            assert abs(wt[2] - rs.p_star) < 1e-9 * rs.p_star
            n_fans += 1
        if rs.p_star < b[2]:
            ar = sound(b[0], b[2])
            head = b[1] + ar
            tail = rs.u_star + sound(b[0] * (rs.p_star / b[2]) ** (1 / G), rs.p_star)
            for xi in np.linspace(tail, head, 7)[1:-1]:
                w, _ = orc.riemann_sample(a, b, rs, xi)
                aw = sound(w[0], w[2])
                assert abs(w[1] - 2 * aw / (G - 1) - (b[1] - 2 * ar / (G - 1))) < 1e-12 * (1 + ar)
                assert abs(w[2] / w[0] ** G - b[2] / b[0] ** G) < 1e-12 * b[2] / b[0] ** G
                assert abs(w[1] + aw - xi) < 1e-12 * (1 + abs(xi))
            n_fans += 1
    assert n_fans > 500


def test_vacuum_generation(orc):
    rho, p = 1.0, 0.4
    a = sound(rho, p)
    U = 2 * a / (G - 1) + 0.5  # separation faster than the escape speed
    rs = orc.riemann_solve([rho, -U, p], [rho, U, p])
    assert rs.vacuum == 1
    w, _ = orc.riemann_sample([rho, -U, p], [rho, U, p], rs, 0.0)
    assert w[0] == 0.0 and w[2] == 0.0
    flux, out = orc.face_flux([rho, -U, 0, 0, p], [rho, U, 0, 0, p], [1.0, 0, 0])
    assert out.vacuum == 1 and np.all(flux == 0.0)


def _euler_flux(w, n):
    rho, u, p = w[0], w[1:4], w[4]
    un = u @ n
    E = p / (G - 1) + 0.5 * rho * (u @ u)
    return np.concatenate([[rho * un], rho * un * u + p * n, [un * (E + p)]])


def test_flux_consistency_rotation_antisymmetry(orc):
    g = np.random.default_rng(6)
    for _ in range(300):
        wl = np.concatenate([[g.uniform(0.2, 3)], g.uniform(-1, 1, 3), [g.uniform(0.2, 3)]])
        wr = np.concatenate([[g.uniform(0.2, 3)], g.uniform(-1, 1, 3), [g.uniform(0.2, 3)]])
        A = g.normal(size=3)
        amag = np.linalg.norm(A)
        # consistency
        f, _ = orc.face_flux(wl, wl, A)
        ref = amag * _euler_flux(wl, A / amag)
        assert np.abs(f - ref).max() < 1e-13 * np.abs(ref).max()
        # rotation equivariance
        Q, r = np.linalg.qr(g.normal(size=(3, 3)))
        Q = Q * np.sign(np.diag(r))
        if np.linalg.det(Q) < 0:
            Q[:, 0] = -Q[:, 0]
        rot = lambda w: np.concatenate([[w[0]], Q @ w[1:4], [w[4]]])
        f1, _ = orc.face_flux(wl, wr, A)
        f2, _ = orc.face_flux(rot(wl), rot(wr), Q @ A)
        back = np.concatenate([[f2[0]], Q.T @ f2[1:4], [f2[4]]])
        assert np.abs(back - f1).max() < 1e-13 * (np.abs(f1).max() + 1)
        # antisymmetry: swapping sides and flipping the normal negates the flux
        f3, _ = orc.face_flux(wr, wl, -A)
        assert np.abs(f3 + f1).max() < 1e-13 * (np.abs(f1).max() + 1)


def test_state_errors(orc):
    with pytest.raises(orc.OracleError) as e:
        orc.riemann_solve([0.0, 0, 1], [1, 0, 1])
    assert e.value.code == orc.E_STATE
    with pytest.raises(orc.OracleError):
        orc.riemann_solve([1.0, 0, -1], [1, 0, 1])
