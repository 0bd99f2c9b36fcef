"""GPU tests of the device-memory hook (tafv_set_allocator): every device
buffer of a context comes from the caller's allocator (here PyTorch's
caching allocator, counted), results are bit-identical to the library's own
hipMalloc, an allocator that returns NULL makes the failing call return
TAFV_E_OOM with every buffer it took handed back, and the context can then
still be used or destroyed without a leak.
"""
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


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available()
    return torch


class Counting:
    """PyTorch caching-allocator memory, counted per pointer; returns NULL
    (0) once `budget` allocations have been made.  Callback errors are
    recorded (an exception cannot cross the C boundary)."""

    def __init__(self, torch, budget=None, misalign=0):
        self.torch = torch
        self.budget = budget
        self.misalign = misalign
        self.live = {}
        self.calls = 0
        self.errors = []

    def alloc(self, n):
        if self.budget is not None and self.calls >= self.budget:
            return 0
        self.calls += 1
        p = self.torch.cuda.caching_allocator_alloc(n + self.misalign, 0)
        self.live[p + self.misalign] = (p, n)
        return p + self.misalign

    def dealloc(self, q):
        if q not in self.live:
            self.errors.append(f"dealloc of unknown pointer {q:#x}")
            return
        p, _ = self.live.pop(q)
        self.torch.cuda.caching_allocator_delete(p)

    @property
    def pair(self):
        return (self.alloc, self.dealloc)


def _small():
    nodes, tets = I.graded_cube_mesh(6, 4.0)
    return nodes, tets, I.blast_state(nodes, tets, centre=I.blast_centre(5))


def test_torch_allocator_same_bits(T, torch):
    """The 12^3 blast at first order and a 6^3 one at second order: the
    same bits with PyTorch's allocator as with hipMalloc; every buffer is
    the allocator's while the context lives, none after."""
    stream = torch.cuda.current_stream().cuda_stream
    cases = [(I.config_small(), 1, 3), (dict(zip(("nodes", "tets", "prim"), _small())), 2, 4)]
    for cfg, order, L in cases:
        res = []
        for use in (False, True):
            a = Counting(torch)
            s = T.Solver(hip_stream=stream, max_levels=L, order=order,
                         allocator=a.pair if use else None)
            s.upload(cfg["nodes"], cfg["tets"])
            s.init(cfg["prim"])
            s.advance(5)
            s.advance(6)
            res.append(s.checkpoint())
            nbuf = T.tafv_device_buffers(s.ctx)
            if use:
                assert nbuf == len(a.live) > 20
            else:
                assert nbuf > 20 and not a.live
            s.close()
            assert not a.live and not a.errors
        for k in ("cons", "accum", "levels"):
            assert np.array_equal(res[0][k], res[1][k]), k
        say(f"order {order}: bit-identical with the caller's allocator ({nbuf} buffers)")


def _workflow(T, torch, a, log):
    """Calls that allocate device memory, in order; stops at the first
    failure and returns its status (0 if none failed)."""
    nodes, tets, prim = _small()
    stream = torch.cuda.current_stream().cuda_stream
    s = T.Solver(hip_stream=stream, max_levels=4, order=2, guess=T.GUESS_MLP, guess_stats=1,
                 allocator=a.pair)
    th = M.he_uniform(3).astype(np.float32)
    x = np.random.default_rng(0).normal(0, 0.1, (300, 6)).astype(np.float32)
    steps = [("upload", lambda: s.upload(nodes, tets)),
             ("mlp_set", lambda: T.tafv_mlp_set(s.ctx, th)),
             ("facelog", lambda: T.tafv_facelog_config(s.ctx, 500, 0.5, 1)),
             ("init", lambda: s.init(prim)),
             ("advance", lambda: s.advance(3)),
             ("mlp_forward", lambda: T.tafv_mlp_forward(s.ctx, x)),
             ("mlp_grad", lambda: T.tafv_mlp_grad(s.ctx, x, x[:, 0].copy())),
             ("mlp_train", lambda: T.tafv_mlp_train(s.ctx, x, x[:, 0].copy(), 2, 128)),
             ("upload2", lambda: s.upload(nodes, tets)),
             ("init2", lambda: s.init(prim, mesh_id=1))]
    code, where = 0, None
    for name, fn in steps:
        try:
            fn()
        except T.TafvError as e:
            code, where = e.code, name
            break
    held = T.tafv_device_buffers(s.ctx)
    log.append((where, held, len(a.live)))
    assert held == len(a.live), (where, held, len(a.live))
    if code == 0:
        st = s.advance(2)
        assert st["cell_updates"] > 0
    s.close()
    return code, where


def test_null_allocation_everywhere(T, torch):
    """Let the n-th allocation of a workflow fail, for every n: the failing
    call returns TAFV_E_OOM, the context holds exactly the buffers the
    allocator still counts, and destroying it returns every one of them."""
    full = Counting(torch)
    log = []
    assert _workflow(T, torch, full, log) == (0, None)
    total = full.calls
    say(f"workflow: {total} device allocations")
    assert total > 40
    seen = set()
    for n in range(total):
        a = Counting(torch, budget=n)
        code, where = _workflow(T, torch, a, log)
        assert code == T.E_OOM, (n, code, where)
        assert not a.live and not a.errors, (n, where, a.live, a.errors)
        seen.add(where)
    say(f"failing calls covered: {sorted(seen)}")
    assert {"upload", "mlp_set", "facelog", "mlp_forward", "mlp_grad", "upload2"} <= seen


def test_null_allocation_batched(T, torch):
    """The batched form merges its meshes and tunes its launches on the
    first state_init and advance: a NULL allocation anywhere there fails the
    call with TAFV_E_OOM and destroying the context returns every buffer."""
    nodes, tets, prim = _small()
    stream = torch.cuda.current_stream().cuda_stream

    def run(a):
        s = T.Solver(hip_stream=stream, max_levels=3, order=2, batch=1, allocator=a.pair)
        code = 0
        try:
            s.upload(nodes, tets)
            s.upload(*I.graded_cube_mesh(4, 2.0))
            T.tafv_batch_config(s.ctx, 1, 1, None)
            s.init(prim, mesh_id=0)
            s.init(I.blast_state(*I.graded_cube_mesh(4, 2.0)), mesh_id=1)
            s.advance(4)
        except T.TafvError as e:
            code = e.code
        assert T.tafv_device_buffers(s.ctx) == len(a.live)
        s.close()
        return code

    full = Counting(torch)
    assert run(full) == 0
    total = full.calls
    say(f"batched workflow: {total} device allocations")
    for n in range(total):
        a = Counting(torch, budget=n)
        assert run(a) == T.E_OOM, n
        assert not a.live and not a.errors, n


def test_context_usable_after_oom(T, torch):
    """A mesh upload that ran out of memory leaves the context as it was:
    with memory available again the same upload and a run succeed, with the
    same bits as a context that never failed."""
    nodes, tets, prim = _small()
    a = Counting(torch, budget=7)
    s = T.Solver(max_levels=4, order=2, allocator=a.pair)
    with pytest.raises(T.TafvError) as e:
        s.upload(nodes, tets)
    assert e.value.code == T.E_OOM
    assert T.tafv_device_buffers(s.ctx) == 0 and not a.live
    a.budget = None
    s.upload(nodes, tets)
    s.init(prim)
    s.advance(7)
    ck = s.checkpoint()
    s.close()
    r = T.Solver(max_levels=4, order=2)
    r.upload(nodes, tets)
    r.init(prim)
    r.advance(7)
    ck2 = r.checkpoint()
    r.close()
    assert np.array_equal(ck["cons"], ck2["cons"]) and np.array_equal(ck["accum"], ck2["accum"])
    assert not a.live and not a.errors


def test_allocator_contract_errors(T, torch):
    nodes, tets, prim = _small()
    a = Counting(torch)
    s = T.Solver(max_levels=3, order=1)
    # one function without the other
    rc = T.lib.tafv_set_allocator(s.ctx, T.ALLOC_FN(lambda n, u: 0), T.DEALLOC_FN(), None)
    assert rc == T.E_ARG
    s.upload(nodes, tets)
    # the context holds memory: the allocator cannot change any more
    with pytest.raises(T.TafvError) as e:
        T.tafv_set_allocator(s.ctx, *a.pair)
    assert e.value.code == T.E_ORDER
    s.close()
    # a misaligned pointer is handed back and the call fails
    b = Counting(torch, misalign=16)
    s = T.Solver(max_levels=3, order=1, allocator=b.pair)
    with pytest.raises(T.TafvError) as e:
        s.upload(nodes, tets)
    assert e.value.code == T.E_DEVICE
    assert not b.live and not b.errors and b.calls >= 1
    s.close()
