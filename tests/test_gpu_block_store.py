"""GPU parity of the block store (Example 1.1): S over a partitioned graph kept as the
blocks' S_Gi plus only the block pairs that the cross-block batch reaches, through the C ABI.
The stored S (materialised) against the oracle's pipeline and against the dense store, the
pairs held against the support of the oracle's Delta S, queries, a further batch, and the
rejections."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import incremental as OI
from oracle import partition as Pt
from oracle import serving as Sv

from _util import EdgeTracker, maxabs

pytestmark = pytest.mark.gpu

C = 0.6


def _say(msg):
    print(msg, flush=True)


def ctx_for(n, s, d, **kw):
    from paper_1711_00121_amd import Context
    return Context(n, s, d, **kw)


def block_pairs(S, lab):
    """Block pairs (p <= q) holding a nonzero entry of S."""
    nb = int(lab.max()) + 1
    out = set()
    for p in range(nb):
        rp = lab == p
        for q in range(p, nb):
            if np.any(S[np.ix_(rp, lab == q)] != 0.0):
                out.add((p, q))
    return out


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("hilo", 1e-6), ("fp32", 1e-6)])
@pytest.mark.parametrize("p_cross", [0.001, 0.03])
def test_block_store_matches_oracle(prec, tol, p_cross):
    """n = 1200 over 16 blocks of scattered ids; with few cross edges (0.1% planted) the
    cross-block Delta S reaches a fraction of the block pairs, with more (3%) all of them.
    The stored S equals the oracle's pipeline (blocks' fixed points, then Inc-bSR of the
    cross edges at K = 15), the dense store's S, and is exactly symmetric; the pairs held
    cover the support of the oracle's Delta S."""
    from paper_1711_00121_amd import partition
    n, m, parts = 1200, 12000, 16
    s, d, _ = W.communities(n, m, parts, p_cross, seed=1102)
    lab = partition(n, s, d, parts)
    _say(f"block store n={n} m={m} p_cross={p_cross} {prec}")
    ref = Pt.partitioned(n, s, d, lab, C, 15)
    ctx = ctx_for(n, s, d, init="partitioned", part=lab, s_prec=prec, K=15, block_store=True)
    S = ctx.S().cpu().numpy()
    err = maxabs(S, ref)
    assert np.array_equal(S, S.T)
    dense = ctx_for(n, s, d, init="partitioned", part=lab, s_prec=prec, K=15)
    gap = maxabs(S, dense.S().cpu().numpy())
    nbytes, npairs = ctx.store_bytes()
    dbytes, _ = dense.store_bytes()
    dense.close()
    inside = lab[s] == lab[d]
    S_old = Pt.block_simrank(n, s[inside], d[inside], lab, C)
    need = block_pairs(ref - S_old, lab) | {(p, p) for p in range(parts)}
    _say(f"max |S - S_oracle| = {err:.3e}, vs dense store {gap:.3e}; {npairs} of "
         f"{parts * (parts + 1) // 2} block pairs held, {nbytes / 8 / n / n:.3f} n^2 entries "
         f"(dense store {dbytes / 8 / n / n:.3f}); oracle Delta S reaches {len(need)} pairs")
    assert err < tol
    assert gap < (1e-12 if prec == "fp64" else 1e-6)
    assert npairs >= len(need)
    # float32 entries (4 B) where the other stores keep 8 B
    assert dbytes == n * ((n + 63) // 64 * 64) * (4 if prec == "fp32" else 8)
    if p_cross < 0.01:
        assert npairs < parts * (parts + 1) // 2 and nbytes < 0.75 * n * n * 8
    ctx.close()


def test_block_store_pairs_held_are_the_reached_pairs():
    """The pairs held are those of the oracle's Delta S support (held pairs whose entries are
    all zero would be wasted memory): equal sets at n = 1200, 0.1% planted cross edges."""
    from paper_1711_00121_amd import partition
    n, m, parts = 1200, 12000, 16
    s, d, _ = W.communities(n, m, parts, 0.001, seed=1102)
    lab = partition(n, s, d, parts)
    ctx = ctx_for(n, s, d, init="partitioned", part=lab, s_prec="fp64", K=15, block_store=True)
    S = ctx.S().cpu().numpy()
    held = block_pairs(S, lab) | {(p, p) for p in range(parts)}
    _, npairs = ctx.store_bytes()
    ref = Pt.partitioned(n, s, d, lab, C, 15)
    inside = lab[s] == lab[d]
    S_old = Pt.block_simrank(n, s[inside], d[inside], lab, C)
    need = block_pairs(ref - S_old, lab) | {(p, p) for p in range(parts)}
    _say(f"pairs held {npairs}, nonzero in S {len(held)}, oracle Delta S {len(need)}")
    assert held == need
    assert npairs == len(need)
    ctx.close()


def test_block_store_queries_match_its_rows():
    """query_column, query_columns, sr_gather_pairs and query_topk read the same S as the
    materialised store; the top-k lists are the oracle's selection of those rows, bit for
    bit."""
    from paper_1711_00121_amd import partition
    n, m, parts = 1500, 15000, 12
    s, d, _ = W.communities(n, m, parts, 0.002, seed=1202)
    lab = partition(n, s, d, parts)
    ctx = ctx_for(n, s, d, init="partitioned", part=lab, s_prec="hilo", K=15, block_store=True)
    S = ctx.S().cpu().numpy()
    xs = np.asarray([0, 7, 311, n - 1], dtype=np.int32)
    for x in xs:
        assert np.array_equal(ctx.query_column(int(x)).cpu().numpy(), S[x])
    cols = ctx.query_columns(xs).cpu().numpy()
    assert np.array_equal(cols, S[xs].astype(np.float32))
    g = np.random.default_rng(5)
    a = g.integers(n, size=5000).astype(np.int32)
    b = g.integers(n, size=5000).astype(np.int32)
    assert np.array_equal(ctx.gather_pairs(a, b).cpu().numpy(), S[a, b])
    q = g.choice(n, 300, replace=False).astype(np.int32)
    for k in (1, 20, 100):
        idx, val = ctx.query_topk(q, k)
        idx, val = idx.cpu().numpy(), val.cpu().numpy()
        for t, x in enumerate(q):
            ri, rv = Sv.topk(S[x], int(x), k)
            assert np.array_equal(idx[t], ri) and np.array_equal(val[t], rv)
    ctx.close()


def test_block_store_takes_further_batches():
    """After the partitioned start, batches of insertions and deletions between existing
    nodes go into the reached pairs (allocating new ones): equal to the dense store given the
    same batches, and to the oracle's Inc-bSR at the same K."""
    from paper_1711_00121_amd import partition
    n, m, parts = 900, 7200, 9
    s, d, _ = W.communities(n, m, parts, 0.001, seed=1302)
    lab = partition(n, s, d, parts)
    kw = dict(init="partitioned", part=lab, s_prec="fp64", K=15,
              edge_cap=m + 400, batch_chunk=8)
    ctx = ctx_for(n, s, d, block_store=True, **kw)
    dense = ctx_for(n, s, d, **kw)
    S_or = Pt.partitioned(n, s, d, lab, C, 15)
    tr = EdgeTracker(n, s, d)
    for step in range(2):
        bi, bj, bo = W.existing_batch(n, *tr.arrays(), n_ins=40, n_del=12, shared=10,
                                      seed=1400 + step)
        cs, cd = tr.arrays()
        S_or, _ = OI.inc_bsr(n, cs, cd, S_or, bi, bj, bo, C, 15)
        before = ctx.store_bytes()[1]
        ctx.apply_batch(bi, bj, bo)
        dense.apply_batch(bi, bj, bo)
        plus, minus = OI.net_update(bi, bj, bo)
        for (i, j) in minus:
            tr.apply(i, j, -1)
        for (i, j) in plus:
            tr.apply(i, j, 1)
        S = ctx.S().cpu().numpy()
        _say(f"batch {step}: pairs held {before} -> {ctx.store_bytes()[1]}; "
             f"vs dense {maxabs(S, dense.S().cpu().numpy()):.3e}, vs oracle "
             f"{maxabs(S, S_or):.3e}")
        assert maxabs(S, dense.S().cpu().numpy()) < 1e-12
        assert maxabs(S, S_or) < 1e-12
        assert np.array_equal(S, S.T)
    assert ctx.sizes() == dense.sizes()
    ctx.close()
    dense.close()


def test_block_store_rejections_leave_state():
    from paper_1711_00121_amd import partition
    from paper_1711_00121_amd._lib import SR_EMODE, SimRankError
    n, m, parts = 300, 2400, 4
    s, d, _ = W.communities(n, m, parts, 0.01, seed=1502)
    lab = partition(n, s, d, parts)
    ctx = ctx_for(n, s, d, init="partitioned", part=lab, s_prec="fp64", K=15, block_store=True,
                  node_cap=n + 8)
    S0 = ctx.S().cpu().numpy()
    held0 = ctx.store_bytes()
    tr = EdgeTracker(n, s, d)
    bi, bj, bo = W.existing_batch(n, *tr.arrays(), n_ins=4, n_del=2, shared=2, seed=1503)
    ins = [(int(a), int(b)) for a, b, o in zip(bi, bj, bo) if o > 0]
    with pytest.raises(SimRankError) as e:
        ctx.apply_edge_update(*ins[0], 1)
    assert e.value.status == SR_EMODE
    # a batch that would create a node (within the node capacity)
    with pytest.raises(SimRankError) as e:
        ctx.apply_batch(np.asarray([0], np.int32), np.asarray([n], np.int32),
                        np.asarray([1], np.int8))
    assert e.value.status == SR_EMODE
    with pytest.raises(SimRankError) as e:
        ctx.backward([0], [1], [1.0])
    assert e.value.status == SR_EMODE
    import ctypes
    qi = np.asarray([0, 1], dtype=np.int32)
    idx = torch.empty((2, 3), dtype=torch.int32, device="cuda")
    val = torch.empty((2, 3), dtype=torch.float64, device="cuda")
    st = ctx.lib.query_topk_noalloc(ctx.h, qi.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                    2, 3, 1, ctypes.c_void_p(idx.data_ptr()),
                                    ctypes.c_void_p(val.data_ptr()))
    assert st == SR_EMODE
    assert np.array_equal(ctx.S().cpu().numpy(), S0)
    assert ctx.store_bytes() == held0 and ctx.sizes() == (n, m)
    ctx.close()
    with pytest.raises(SimRankError) as e:
        ctx_for(n, s, d, block_store=True)
    assert e.value.status == SR_EMODE
    # the pair table holds labels below 4096
    from paper_1711_00121_amd._lib import SR_ECAPACITY
    big = 4100
    bs_, bd_ = W.chung_lu(big, 8000, seed=1504)
    with pytest.raises(SimRankError) as e:
        ctx_for(big, bs_, bd_, init="partitioned", part=np.arange(big, dtype=np.int32),
                block_store=True)
    assert e.value.status == SR_ECAPACITY
    torch.cuda.synchronize()
