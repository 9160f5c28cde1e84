"""query_topk_noalloc, the variant of query_topk that allocates nothing (the query ids are
staged in a static per-GPU device array), called through the C ABI: its output equals
query_topk's bit for bit on two calls in a row, the second with fewer queries, in dense and
column mode; more queries than the array holds are refused before any work."""
import ctypes as C

import numpy as np
import pytest
import torch

import workloads as W
from paper_1711_00121_amd import Context
from paper_1711_00121_amd import _lib as L

pytestmark = pytest.mark.gpu

MAX_IDS = 65536


def noalloc_topk(ctx, q, k, exclude_self=True):
    q = np.ascontiguousarray(np.asarray(q, dtype=np.int32))
    idx = torch.full((len(q), k), -7, dtype=torch.int32, device="cuda")
    val = torch.full((len(q), k), -7.0, dtype=torch.float64, device="cuda")
    st = L.load().query_topk_noalloc(ctx.h, q.ctypes.data_as(C.POINTER(C.c_int32)), len(q),
                                     int(k), int(bool(exclude_self)), C.c_void_p(idx.data_ptr()),
                                     C.c_void_p(val.data_ptr()))
    torch.cuda.synchronize()
    return st, idx, val


def check_two_calls(ctx, n, seed):
    g = np.random.default_rng(seed)
    for nq, k in ((700, 100), (130, 17)):
        q = g.integers(0, n, size=nq).astype(np.int32)
        st, idx, val = noalloc_topk(ctx, q, k)
        assert st == L.SR_OK
        ref_idx, ref_val = ctx.query_topk(q, k)
        torch.cuda.synchronize()
        assert torch.equal(idx, ref_idx), (nq, k)
        assert torch.equal(val, ref_val), (nq, k)


def test_noalloc_topk_dense_matches_query_topk():
    n = 3000
    s, d = W.chung_lu(n, 15000, seed=961)
    batches, counts = W.batch_stream(n, s, d, 1, 300, seed=962)
    ctx = Context(n, s, d, C=0.6, K=10, s_prec="hilo", node_cap=counts[0])
    bi, bj, bo = batches[0]
    ctx.apply_batch(bi, bj, bo)
    check_two_calls(ctx, ctx.sizes()[0], 963)
    ctx.close()


def test_noalloc_topk_column_mode_matches_query_topk():
    n = 2000
    s, d = W.chung_lu(n, 10000, seed=964)
    ctx = Context(n, s, d, C=0.6, K=10, K_ps=20, mode="column")
    g = np.random.default_rng(965)
    for nq, k in ((9, 40), (4, 5)):
        q = g.integers(0, n, size=nq).astype(np.int32)
        st, idx, val = noalloc_topk(ctx, q, k)
        assert st == L.SR_OK
        ref_idx, ref_val = ctx.query_topk(q, k)
        torch.cuda.synchronize()
        assert torch.equal(idx, ref_idx) and torch.equal(val, ref_val), (nq, k)
    ctx.close()


def test_noalloc_topk_refuses_more_ids_than_the_array_holds():
    n = 500
    s, d = W.chung_lu(n, 2000, seed=966)
    ctx = Context(n, s, d, C=0.6, K=8, s_prec="fp64")
    q = np.zeros(MAX_IDS + 1, dtype=np.int32)
    st, idx, val = noalloc_topk(ctx, q, 3)
    assert st == L.SR_ECAPACITY
    assert bool((idx == -7).all()) and bool((val == -7.0).all())
    st, idx, val = noalloc_topk(ctx, [n], 3)
    assert st == L.SR_ERANGE
    # a full array is accepted and still matches
    q = np.arange(MAX_IDS, dtype=np.int32) % n
    st, idx, val = noalloc_topk(ctx, q, 3)
    assert st == L.SR_OK
    ref_idx, ref_val = ctx.query_topk(q, 3)
    assert torch.equal(idx, ref_idx) and torch.equal(val, ref_val)
    ctx.close()
