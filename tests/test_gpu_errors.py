"""The boundary's error promise: a validation error (status code) leaves the context as it
was, and a refused call launches nothing. Each case is forced from the host."""
import numpy as np
import pytest
import torch

import workloads as W
from paper_1711_00121_amd import Context, simrank_pairs
from paper_1711_00121_amd import _lib as L

from _util import maxabs

pytestmark = pytest.mark.gpu

C = 0.6


def status_of(fn, *a, **k):
    try:
        fn(*a, **k)
    except L.SimRankError as e:
        return e.status
    return L.SR_OK


def snapshot(ctx):
    return ctx.sizes(), ctx.S().cpu().numpy().copy()


def assert_unchanged(ctx, snap):
    sizes, S = snap
    assert ctx.sizes() == sizes
    assert np.array_equal(ctx.S().cpu().numpy(), S)


def test_node_capacity_leaves_context_unchanged():
    n = 120
    s, d = W.chung_lu(n, 500, seed=901)
    ctx = Context(n, s, d, C=C, K=8, s_prec="fp64", node_cap=n)
    snap = snapshot(ctx)
    # C1 (new sink), C2 (new source) and C3 all need a node past the capacity
    for i, j in [(3, n), (n, 4), (n, n + 1)]:
        assert status_of(ctx.apply_edge_update, i, j, 1) == L.SR_ECAPACITY
        assert_unchanged(ctx, snap)
    assert status_of(ctx.apply_batch, [1, 2, n], [n, 5, 6], [1, 1, 1]) == L.SR_ECAPACITY
    assert_unchanged(ctx, snap)
    # the context still works
    es = set(zip(s.tolist(), d.tolist()))
    i, j = next((a, b) for a in range(n) for b in range(n) if a != b and (a, b) not in es)
    ctx.apply_edge_update(i, j, 1)
    assert ctx.sizes() == (n, len(s) + 1)
    ctx.close()


def test_edge_capacity_leaves_context_unchanged():
    n = 120
    s, d = W.chung_lu(n, 500, seed=902)
    ctx = Context(n, s, d, C=C, K=8, s_prec="fp64", node_cap=n + 4, edge_cap=len(s) + 2)
    es = set(zip(s.tolist(), d.tolist()))
    free = [(a, b) for a in range(n) for b in range(n) if a != b and (a, b) not in es]
    ctx.apply_edge_update(*free[0], 1)
    ctx.apply_edge_update(*free[1], 1)
    snap = snapshot(ctx)
    assert status_of(ctx.apply_edge_update, *free[2], 1) == L.SR_ECAPACITY
    assert_unchanged(ctx, snap)
    assert status_of(ctx.apply_edge_update, 5, n, 1) == L.SR_ECAPACITY
    assert_unchanged(ctx, snap)
    bi = [free[3][0], free[4][0]]
    bj = [free[3][1], free[4][1]]
    assert status_of(ctx.apply_batch, bi, bj, [1, 1]) == L.SR_ECAPACITY
    assert_unchanged(ctx, snap)
    # a deletion then fits again
    ctx.apply_edge_update(*free[0], -1)
    ctx.apply_edge_update(*free[2], 1)
    assert ctx.sizes() == (n, len(s) + 2)
    ctx.close()


def test_validation_errors_leave_context_unchanged():
    n = 100
    s, d = W.chung_lu(n, 400, seed=903)
    ctx = Context(n, s, d, C=C, K=8, s_prec="hilo", node_cap=n + 8)
    snap = snapshot(ctx)
    e0 = (int(s[0]), int(d[0]))
    es = set(zip(s.tolist(), d.tolist()))
    free = next((a, b) for a in range(n) for b in range(n) if a != b and (a, b) not in es)
    cases = [
        (ctx.apply_edge_update, (e0[0], e0[1], 1), L.SR_EEXIST),
        (ctx.apply_edge_update, (free[0], free[1], -1), L.SR_ENOENT),
        (ctx.apply_edge_update, (4, 4, 1), L.SR_ESELF),
        (ctx.apply_edge_update, (3, n + 1, 1), L.SR_ERANGE),
        (ctx.apply_edge_update, (3, 5, 2), L.SR_EINVAL),
        (ctx.apply_batch, ([e0[0], free[0]], [e0[1], free[1]], [1, 1]), L.SR_EEXIST),
        (ctx.apply_batch, ([free[0]], [free[1]], [-1]), L.SR_ENOENT),
        (ctx.apply_batch, ([free[0], free[0]], [free[1], free[1]], [1, 1]), L.SR_EEXIST),
        (ctx.apply_batch, ([1, 2], [n + 1, 3], [1, 1]), L.SR_ERANGE),   # new ids not dense
        (ctx.apply_batch, ([2], [2], [1]), L.SR_ESELF),
    ]
    for fn, args, want in cases:
        assert status_of(fn, *args) == want, (fn.__name__, args)
        assert_unchanged(ctx, snap)
    ctx.close()


def test_out_of_memory_at_init_then_a_working_context():
    """A node capacity whose dense S cannot be allocated (300k x 300k x 8 B = 720 GB) is
    SR_ENOMEM; the failed allocation leaves no error behind for the next context."""
    n = 60
    s, d = W.chung_lu(n, 200, seed=904)
    assert status_of(Context, n, s, d, C=C, K=8, s_prec="fp64", node_cap=300_000) == \
        L.SR_ENOMEM
    ctx = Context(n, s, d, C=C, K=8, s_prec="fp64", node_cap=n + 2)
    ctx.apply_edge_update(3, n, 1)
    ctx.apply_batch([n + 1], [5], [1])
    assert ctx.sizes()[0] == n + 2
    ctx.close()


def test_pair_ids_out_of_range_are_refused():
    n = 80
    s, d = W.chung_lu(n, 300, seed=905)
    w = W.lognormal_weights(len(s), seed=906)
    ctx = Context(n, s, d, weight=w, C=C, K=8, s_prec="fp64")
    good = ctx.gather_pairs([1, 2], [3, 4])
    for a, b in ([[1, n], [3, 4]], [[1, 2], [-1, 4]], [[n + 7], [0]]):
        assert status_of(ctx.gather_pairs, a, b) == L.SR_ERANGE
        g = torch.ones(len(a), dtype=torch.float64, device="cuda")
        assert status_of(ctx.backward, a, b, g) == L.SR_ERANGE
    assert torch.equal(ctx.gather_pairs([1, 2], [3, 4]), good)
    # and the context still differentiates
    dw = ctx.backward([1, 2], [3, 4], torch.ones(2, dtype=torch.float64, device="cuda"))
    assert dw.shape == (len(s),) and torch.isfinite(dw).all()
    ctx.close()


def test_simrank_pairs_refuses_other_weights():
    n = 80
    s, d = W.chung_lu(n, 300, seed=907)
    w = W.lognormal_weights(len(s), seed=908)
    ctx = Context(n, s, d, weight=w, C=C, K=8, s_prec="fp64")
    wt = torch.tensor(w, dtype=torch.float64, device="cuda", requires_grad=True)
    v = simrank_pairs(wt, ctx, [1, 2], [3, 4])
    v.sum().backward()
    assert wt.grad is not None and wt.grad.shape == (len(s),)
    w2 = wt.detach().clone()
    w2[5] *= 1.5
    with pytest.raises(ValueError):
        simrank_pairs(w2.requires_grad_(), ctx, [1, 2], [3, 4])
    ctx.close()
