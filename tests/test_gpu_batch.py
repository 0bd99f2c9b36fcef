"""GPU tests of the batched form (params.batch = 1): many meshes with their
own level caps and staggered schedules advanced by one fixed launch
sequence per subiteration.

  * parity: each mesh of a mixed batch against the FP64 oracle run on that
    mesh alone (normwise <= 1e-12 on cons + accum / V, the state at the end
    of each cell's current step; identical levels and schedule counters);
  * the batch equals the same meshes advanced one after another by the
    single-mesh path, bit for bit, in FP32 with the learned guess;
  * HIP-graph replays equal direct launches, bit for bit, call after call,
    with host reads in between; the autotuner's choice and its cache file;
  * the batched workload at full size (128 meshes): the three smallest and
    three largest meshes and the largest mesh at the highest level cap
    against the oracle in FP64, and FP32 + learned guess against FP64 by
    L1 error on every mesh;
  * error codes of the batched calls.
"""
import os
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
    scale = np.abs(b).max(0)
    scale[scale == 0] = 1.0
    return (np.abs(a - b).max(0) / scale).max()


def volumes(nodes, tets):
    p = nodes[tets]
    return np.einsum("ij,ij->i", p[:, 1] - p[:, 0],
                     np.cross(p[:, 2] - p[:, 0], p[:, 3] - p[:, 0])) / 6.0


def l1_rel(a, b, vol):
    return (vol * np.abs(a - b)).sum() / (vol * np.abs(b)).sum()


def mixed_cases():
    """Meshes of uneven size, grading and level cap, with a one-hex mesh
    (6 tets) and a single-level mesh among them."""
    out = []
    nodes, tets = I.graded_box_mesh(6, 6, 4, 8.0)
    out.append((nodes, tets, I.blast_state(nodes, tets, centre=I.blast_centre(11)), 4))
    nodes, tets = I.graded_cube_mesh(10, 4.0)
    out.append((nodes, tets, I.blast_state(nodes, tets), 1))
    nodes, tets = I.graded_cube_mesh(1, 1.0)
    out.append((nodes, tets, I.random_state(len(tets), 5), 3))
    nodes, tets = I.graded_box_mesh(9, 7, 3, 16.0)
    out.append((nodes, tets, I.blast_state(nodes, tets, centre=I.blast_centre(12)), 6))
    return out


def make_batch(T, cases, graph=1, autotune=1, cache=None, **params):
    s = T.Solver(batch=1, **params)
    for nodes, tets, _, L in cases:
        s.upload(nodes, tets, max_levels=L)
    T.tafv_batch_config(s.ctx, graph, autotune, cache)
    for k, (_, _, prim, _) in enumerate(cases):
        s.init(prim, mesh_id=k)
    return s


@pytest.mark.parametrize("order", [1, 2])
def test_batch_matches_oracle(T, orc, order):
    cases = mixed_cases()
    s = make_batch(T, cases, order=order)
    chunks = [5, 11]
    say(f"batch: {len(cases)} meshes, cells {[len(c[1]) for c in cases]}, order {order}, "
        f"advance {chunks}")
    tot = {"cell_updates": 0, "face_solves": 0}
    for n in chunks:
        st = s.advance(n)
        for k in tot:
            tot[k] += st[k]
    info = T.tafv_batch_info(s.ctx)
    say(f"launch settings: {info}")
    sum_upd = sum_faces = 0
    for k, (nodes, tets, prim, L) in enumerate(cases):
        ck = s.checkpoint(k)
        lev = ck["levels"]
        gs = s.stats(k)
        om = orc.Mesh(nodes, tets)
        o = orc.State(om, prim, orc.params(max_levels=L, order=order))
        for n in chunks:
            o.advance(n)
        u_o, r_o, lev_o = o.read()
        os_ = o.stats()
        vol = om.geometry()["vol"][:, None]
        err = normwise(ck["cons"] + ck["accum"] / vol, u_o + r_o / vol)
        say(f"  mesh {k}: cells {len(tets)} L {L} err {err:.2e} theta {gs['theta']} "
            f"phase {gs['phase']} updates {gs['cell_updates']} / {os_['cell_updates']}")
        assert err <= TOL
        assert (lev == lev_o).all()
        assert gs["cell_updates"] == os_["cell_updates"]
        assert gs["face_solves"] == os_["face_solves"]
        assert gs["phase"] == os_["phase"] and gs["theta"] == os_["theta"]
        sum_upd += gs["cell_updates"]
        sum_faces += gs["face_solves"]
    assert tot["cell_updates"] == sum_upd and tot["face_solves"] == sum_faces
    s.close()


def test_batch_equals_separate_meshes_fp32_learned(T):
    cases = mixed_cases()
    th = (M.he_uniform(3) + np.random.default_rng(4).normal(0, 0.05, M.N_PARAMS)).astype(np.float32)
    common = dict(order=2, precision=T.FP32_FLUX, guess=T.GUESS_MLP, guess_stats=1,
                  guess_gate=0.0)
    s1 = T.Solver(**common)
    for nodes, tets, _, L in cases:
        s1.upload(nodes, tets, max_levels=L)
    T.tafv_mlp_set(s1.ctx, th)
    for k, c in enumerate(cases):
        s1.init(c[2], mesh_id=k)
    s2 = T.Solver(batch=1, **common)
    for nodes, tets, _, L in cases:
        s2.upload(nodes, tets, max_levels=L)
    T.tafv_mlp_set(s2.ctx, th)
    for k, c in enumerate(cases):
        s2.init(c[2], mesh_id=k)
    st1 = s1.advance(16)
    st2 = s2.advance(16)
    for k in range(len(cases)):
        c1, l1 = s1.read(k)
        c2, l2 = s2.read(k)
        assert np.array_equal(c1, c2), k
        assert np.array_equal(l1, l2), k
    for key in ("cell_updates", "face_solves", "newton_updates", "guess_faces", "guess_used",
                "guess_newton_updates"):
        assert st1[key] == st2[key], (key, st1[key], st2[key])
    say(f"fp32 + learned, batch = separate: {st2['cell_updates']} updates, network start on "
        f"{st2['guess_used']} of {st2['guess_faces']} shock faces")
    assert st2["guess_used"] > 0
    s1.close()
    s2.close()


def test_graph_replay_matches_eager(T, tmp_path):
    cases = mixed_cases()
    cache = str(tmp_path / "tune.txt")
    sg = make_batch(T, cases, graph=1, autotune=1, cache=cache)
    se = make_batch(T, cases, graph=0, autotune=0)
    for call in range(4):
        n = 8 if call < 3 else 5
        sg.advance(n)
        se.advance(n)
        for k in range(len(cases)):
            cg, lg = sg.read(k)
            ce, le = se.read(k)
            assert np.array_equal(cg, ce), (call, k)
            assert np.array_equal(lg, le), (call, k)
    info = T.tafv_batch_info(sg.ctx)
    say(f"graph context settings: {info}; eager context: {T.tafv_batch_info(se.ctx)}")
    assert info["source"] == "tuned"
    assert os.path.exists(cache)
    lines = open(cache).read().split("\n")
    assert any(l.strip() for l in lines)
    # a new context with the same key reads the cache instead of timing
    s3 = make_batch(T, cases, graph=1, autotune=1, cache=cache)
    s3.advance(8)
    info3 = T.tafv_batch_info(s3.ctx)
    assert info3["source"] == "cache"
    assert info3["grad"] == info["grad"] and info3["cells"] == info["cells"]
    c3, _ = s3.read(0)
    s4 = make_batch(T, cases, graph=0, autotune=0)
    s4.advance(8)
    c4, _ = s4.read(0)
    assert np.array_equal(c3, c4)
    for s in (sg, se, s3, s4):
        s.close()


def test_reset_and_mesh_params(T):
    cases = mixed_cases()
    s = make_batch(T, cases)
    s.advance(7)
    a = [s.read(k)[0] for k in range(len(cases))]
    for k in range(len(cases)):
        s.reset(k)
    s.advance(7)
    b = [s.read(k)[0] for k in range(len(cases))]
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    T.tafv_state_reset(s.ctx, -1)  # every mesh at once
    s.advance(7)
    for k, x in enumerate(a):
        assert np.array_equal(x, s.read(k)[0])
    # a new level cap takes effect at the mesh's next iteration start
    T.tafv_mesh_params(s.ctx, 0, 1)
    for k in range(len(cases)):
        s.reset(k)
    s.advance(4)
    assert s.stats(0)["theta"] == 0
    s.close()


def test_batch_errors(T):
    with pytest.raises(T.TafvError) as e:
        T.Solver(batch=1, scatter=T.SCATTER_COLOUR)
    assert e.value.code == T.E_ARG
    cases = mixed_cases()[:2]
    s = T.Solver(batch=1)
    for nodes, tets, _, L in cases:
        s.upload(nodes, tets, max_levels=L)
    with pytest.raises(T.TafvError) as e:
        s.advance(1)
    assert e.value.code == T.E_ORDER
    s.init(cases[0][2], mesh_id=0)
    with pytest.raises(T.TafvError) as e:
        s.advance(1)  # mesh 1 has no state
    assert e.value.code == T.E_ORDER
    with pytest.raises(T.TafvError) as e:
        s.upload(cases[0][0], cases[0][1])
    assert e.value.code == T.E_ORDER
    n0 = len(cases[0][1])
    with pytest.raises(T.TafvError) as e:
        T.tafv_checkpoint_write(s.ctx, 0, np.zeros((n0, 5)), np.zeros((n0, 5)),
                                np.zeros(n0, np.int8), 0, 0, 1.0, 0.0)
    assert e.value.code == T.E_ARG
    with pytest.raises(T.TafvError) as e:
        T.tafv_facelog_config(s.ctx, 100, 0.5, 1)
    assert e.value.code == T.E_ARG
    bad = cases[1][2].copy()
    bad[3, 0] = -1.0
    with pytest.raises(T.TafvError) as e:
        s.init(bad, mesh_id=1)
    assert e.value.code == T.E_STATE
    s.close()
    s = T.Solver()
    with pytest.raises(T.TafvError) as e:
        T.tafv_batch_config(s.ctx, 1, 1, None)
    assert e.value.code == T.E_ARG
    s.close()


@pytest.fixture(scope="module")
def full_batch():
    cases = I.config_batch(128)
    say(f"batched workload: {len(cases)} meshes, {sum(len(c['tets']) for c in cases)} cells")
    return cases


def _run_full(T, cases, **params):
    s = T.Solver(batch=1, **params)
    for c in cases:
        s.upload(c["nodes"], c["tets"], max_levels=c["max_levels"])
    return s


@pytest.fixture(scope="module")
def full_fp64(T, full_batch):
    """The batched workload in FP64 with the two-rarefaction start, 16 units."""
    s = _run_full(T, full_batch, order=2)
    for k, c in enumerate(full_batch):
        s.init(c["prim"], mesh_id=k)
    st = s.advance(16)
    say(f"full batch FP64: {st['cell_updates']} cell updates, {st['face_solves']} face solves, "
        f"settings {T.tafv_batch_info(s.ctx)}")
    out = dict(stats=st, cons=[], accum=[], levels=[], mesh_stats=[])
    for k in range(len(full_batch)):
        ck = s.checkpoint(k)
        out["cons"].append(ck["cons"])
        out["accum"].append(ck["accum"])
        out["levels"].append(ck["levels"])
        out["mesh_stats"].append(s.stats(k))
    s.close()
    return out


def full_batch_sample(cases):
    """The three smallest and the three largest meshes, and the largest
    mesh with the highest level cap (the largest merged offsets, tile
    prefixes and level counts of the batch)."""
    size = np.array([len(c["tets"]) for c in cases])
    order = np.argsort(size)
    cap = max(c["max_levels"] for c in cases)
    top_cap = max((k for k, c in enumerate(cases) if c["max_levels"] == cap), key=lambda k: size[k])
    return list(dict.fromkeys([*order[:3], *order[-3:], top_cap]))


def test_full_batch_fp64_against_oracle_sample(orc, full_batch, full_fp64):
    for k in full_batch_sample(full_batch):
        c = full_batch[k]
        om = orc.Mesh(c["nodes"], c["tets"])
        o = orc.State(om, c["prim"], orc.params(max_levels=c["max_levels"], order=2))
        o.advance(16)
        u_o, r_o, lev_o = o.read()
        vol = om.geometry()["vol"][:, None]
        err = normwise(full_fp64["cons"][k] + full_fp64["accum"][k] / vol, u_o + r_o / vol)
        say(f"  mesh {k}: {len(c['tets'])} cells, L {c['max_levels']}, err {err:.2e}")
        assert err <= TOL
        assert (full_fp64["levels"][k] == lev_o).all()
        ms, os_ = full_fp64["mesh_stats"][k], o.stats()
        for key in ("cell_updates", "face_solves", "theta", "phase"):
            assert ms[key] == os_[key], (k, key, ms[key], os_[key])


def test_full_batch_fp32_learned_l1(T, full_batch, full_fp64):
    th = M.he_uniform(5).astype(np.float32)
    s = _run_full(T, full_batch, order=2, precision=T.FP32_FLUX, guess=T.GUESS_MLP,
                  guess_gate=0.0)
    T.tafv_mlp_set(s.ctx, th)
    for k, c in enumerate(full_batch):
        s.init(c["prim"], mesh_id=k)
    st = s.advance(16)
    worst = 0.0
    for k, c in enumerate(full_batch):
        a, _ = s.read(k)
        b = full_fp64["cons"][k]
        vol = volumes(c["nodes"], c["tets"])
        e = max(l1_rel(a[:, 0], b[:, 0], vol), l1_rel(a[:, 4], b[:, 4], vol))
        worst = max(worst, e)
    say(f"full batch FP32 + learned: worst per-mesh L1 (rho, E) vs FP64 {worst:.2e}; network "
        f"start on {st['guess_used']} faces")
    assert worst <= 1e-5
    s.close()
