"""The network gradient that allocates no device memory
(tafv_mlp_grad_noalloc, for callers that cannot allocate) against the
allocating tafv_mlp_grad on the same inputs: the same kernels in the same
order, so the gradient and the loss are bit-identical; two calls in a row,
the second with fewer rows, so that nothing left in the shared scratch by
the first call reaches the second; the row limit is enforced; and the call
takes no buffer from the context's allocator."""
import sys

import numpy as np
import pytest

from oracle import mlp_ref as M

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def T():
    from paper_1704_01144_amd import tafv
    return tafv


def _rows(n, seed):
    g = np.random.default_rng(seed)
    x = g.normal(0, 0.2, (n, 6)).astype(np.float32)
    t = g.normal(0, 0.05, n).astype(np.float32)
    return x, t


def test_noalloc_gradient_equals_allocating_gradient(T):
    import torch
    calls = []

    def alloc(nbytes):  # PyTorch memory, every request recorded
        calls.append(nbytes)
        return torch.cuda.caching_allocator_alloc(nbytes, 0)

    s = T.Solver(max_levels=2, order=1, allocator=(alloc, torch.cuda.caching_allocator_delete))
    th = (M.he_uniform(8) + np.random.default_rng(9).normal(0, 0.05, M.N_PARAMS)).astype(np.float32)
    T.tafv_mlp_set(s.ctx, th)
    n_set = len(calls)  # the network's own buffers
    ref = T.Solver(max_levels=2, order=1)
    T.tafv_mlp_set(ref.ctx, th)
    for n, seed in ((T.MLP_GRAD_NOALLOC_MAX_ROWS, 1), (5000, 2), (77, 3)):
        x, t = _rows(n, seed)
        held = T.tafv_device_buffers(s.ctx)
        g0, l0 = T.tafv_mlp_grad_noalloc(s.ctx, x, t)
        assert T.tafv_device_buffers(s.ctx) == held and len(calls) == n_set
        g1, l1 = T.tafv_mlp_grad(ref.ctx, x, t)
        say(f"rows {n}: max |diff| {np.abs(g0 - g1).max():.1e}, loss {l0:.6e} / {l1:.6e}")
        assert np.array_equal(g0, g1) and l0 == l1
    with pytest.raises(T.TafvError) as e:
        T.tafv_mlp_grad_noalloc(s.ctx, *_rows(T.MLP_GRAD_NOALLOC_MAX_ROWS + 1, 4))
    assert e.value.code == T.E_ARG
    assert len(calls) == n_set
    s.close()
    ref.close()


def test_noalloc_gradient_needs_a_network(T):
    s = T.Solver(max_levels=2, order=1)
    with pytest.raises(T.TafvError) as e:
        T.tafv_mlp_grad_noalloc(s.ctx, *_rows(10, 5))
    assert e.value.code == T.E_MLP
    s.close()
