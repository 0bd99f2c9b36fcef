"""GPU tests of the grouped advance (tafv_advance_group): several contexts,
each with its own stream, advanced together by host workers that enqueue one
subiteration of each context in turn.  The arithmetic of every context is
that of its own tafv_advance, so the states, accumulators, levels and
counters equal those of the contexts advanced one after another, bit for
bit, whatever the number of workers and streams; and the arguments are
checked."""
import sys

import numpy as np
import pytest

from paper_1704_01144_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def T():
    from paper_1704_01144_amd import tafv
    return tafv


def cases():
    """Meshes of uneven size, grading and level cap (their iterations start
    at different subiterations)."""
    out = []
    for k, (n, g, L) in enumerate([(10, 16.0, 5), (6, 4.0, 3), (12, 8.0, 4), (3, 1.0, 2),
                                   (8, 32.0, 6)]):
        nodes, tets = I.graded_cube_mesh(n, g)
        out.append((nodes, tets, I.blast_state(nodes, tets, centre=I.blast_centre(20 + k)), L))
    return out


def make(T, torch, cs, streams, **params):
    ss = []
    for k, (nodes, tets, prim, L) in enumerate(cs):
        st = streams[k % len(streams)].cuda_stream if streams else None
        s = T.Solver(hip_stream=st, max_levels=L, **params)
        s.upload(nodes, tets)
        s.init(prim)
        ss.append(s)
    return ss


@pytest.mark.parametrize("workers,nstreams,order,precision",
                         [(1, 1, 2, 0), (2, 3, 2, 0), (5, 5, 2, 1), (3, 2, 1, 0)])
def test_group_equals_separate(T, workers, nstreams, order, precision):
    import torch
    cs = cases()
    streams = [torch.cuda.Stream() for _ in range(nstreams)]
    ref = make(T, torch, cs, None, order=order, precision=precision)
    grp = make(T, torch, cs, streams, order=order, precision=precision)
    chunks = [5, 11, 16]
    tot = 0
    for n in chunks:
        for s in ref:
            s.advance(n)
        st = T.tafv_advance_group([s.ctx for s in grp], n, workers)
        tot += st["cell_updates"]
    torch.cuda.synchronize()
    upd = 0
    for k, (a, b) in enumerate(zip(ref, grp)):
        ca, cb = a.checkpoint(), b.checkpoint()
        for key in ("cons", "accum", "levels"):
            assert np.array_equal(ca[key], cb[key]), (k, key)
        sa, sb = a.stats(), b.stats()
        for key in ("cell_updates", "face_solves", "newton_updates", "theta", "phase",
                    "subiterations"):
            assert sa[key] == sb[key], (k, key)
        assert sa["t_reached"] == sb["t_reached"]
        upd += sb["cell_updates"]
    assert tot == upd
    say(f"workers {workers}, streams {nstreams}, order {order}, precision {precision}: "
        f"{len(cs)} meshes bit-identical, {upd} cell updates")
    for s in ref + grp:
        s.close()


def test_group_arguments(T):
    cs = cases()[:2]
    a = make(T, None, cs, None)
    with pytest.raises(T.TafvError) as e:
        T.tafv_advance_group([a[0].ctx, a[0].ctx], 2, 2)
    assert e.value.code == T.E_ARG
    with pytest.raises(T.TafvError) as e:
        T.tafv_advance_group([a[0].ctx, a[1].ctx], 2, 0)
    assert e.value.code == T.E_ARG
    b = T.Solver(max_levels=3)
    b.upload(cs[0][0], cs[0][1])  # no state
    with pytest.raises(T.TafvError) as e:
        T.tafv_advance_group([a[0].ctx, b.ctx], 2, 2)
    assert e.value.code == T.E_ORDER
    for s in a + [b]:
        s.close()
