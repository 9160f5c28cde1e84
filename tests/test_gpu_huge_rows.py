"""Parity on graphs whose rows exceed the traversals' chunking threshold.

With split_rows = 16,384, a row of more than 16,384 entries is cut into chunks of 8,192
entries, one workgroup per chunk, and a second launch adds the chunks' partial sums; a row of
2,049 to 16,384 entries takes one whole workgroup. The graph here is a Chung-Lu graph
(n = 26,000) with two hubs: H1 with 24,575 in-neighbours (three chunks, one entry short of
the chunk table's cover) and 20,000 out-neighbours, and H2 with 16,384 in-neighbours (the
last length of the whole-workgroup tier). The updates make H1's in-list outgrow its chunk table, move H2 into
the chunked tier and back, and run the column method over H1's chunked out-list.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import graph as Gr
from oracle import incremental as OI
from oracle import simrank as O

from _util import EdgeTracker, maxabs

C = 0.6
N = 26_000
H1, H2 = 5, 7
IN1, OUT1, IN2, OUT2 = 3 * 8192 - 1, 20_000, 16_384, 100
SPLIT = 16_384


def _say(*a):
    print(*a, flush=True)


def _graph():
    s, d = W.chung_lu(N, 4 * N, seed=7001)
    return W.with_hubs(N, s, d, [(H1, IN1, OUT1), (H2, IN2, OUT2)], seed=7002)


def _non_in_neighbours(s, d, h, k, seed):
    """k nodes, other than the hubs, that have no edge into h."""
    have = np.zeros(N, bool)
    have[s[d == h]] = True
    have[[H1, H2]] = True
    return W.rng(seed).choice(np.nonzero(~have)[0], size=k, replace=False).astype(int).tolist()


def _ctx(*a, **kw):
    from paper_1711_00121_amd import Context
    return Context(*a, **kw)


def _check_columns(ctx, Q, cols, bar):
    worst = 0.0
    for x in cols:
        ref = O.single_source(Q, int(x), C, tol=1e-13)
        got = ctx.query_column(int(x)).cpu().numpy()
        worst = max(worst, maxabs(got, ref))
    assert worst < bar, worst
    return worst


@pytest.mark.gpu
def test_huge_rows_stream_pruned():
    s, d = _graph()
    a, b, c = _non_in_neighbours(s, d, H1, 3, seed=7003)
    ctx = _ctx(N, s, d, C=C, K=15, s_prec="hilo", prune=True, split_rows=SPLIT)
    tr = EdgeTracker(N, s, d)
    Q0 = tr.Q()
    e2 = int(s[d == H2][0])  # an existing in-edge of H2
    seq = [(a, H1, 1),   # H1: 24,576 entries, inside its chunk table
           (b, H1, 1),   # 24,577: the table is rebuilt with a fourth chunk
           (c, H2, 1),   # H2: 16,385 entries, into the chunked tier
           (e2, H2, -1),  # back to 16,384, the whole-workgroup tier
           (a, H1, -1)]
    cols = W.column_sample(N, 3, seed=7004, extra=[H1, H2, a, b, c])
    for t, (i, j, op) in enumerate(seq):
        _say(f"huge rows, stream: update {t} ({i}, {j}, {op:+d})")
        ctx.apply_edge_update(i, j, op)
        tr.apply(i, j, op)
        Q = tr.Q()
        if t == 0:
            # Theorem 4: Delta S vanishes outside A_hat x B_hat u B_hat x A_hat
            A, B = (x.cpu().numpy() for x in ctx.get_aff())
            inA = np.zeros(N, bool)
            inB = np.zeros(N, bool)
            inA[A] = True
            inB[B] = True
            for x in cols:
                dS = O.single_source(Q, int(x), C, tol=1e-13) - O.single_source(
                    Q0, int(x), C, tol=1e-13)
                inside = (inA & inB[x]) | (inB & inA[x])
                assert np.abs(dS[~inside]).max(initial=0.0) < 1e-11
        w = _check_columns(ctx, Q, cols, 1e-6)
        _say(f"  max |S_gpu - S*| over {len(cols)} columns = {w:.3e}")
    ctx.close()


@pytest.mark.gpu
def test_huge_rows_column_mode():
    s, d = _graph()
    (i,) = _non_in_neighbours(s, d, H1, 1, seed=7005)
    K, Kps = 10, 30
    block = W.column_sample(N, 61, seed=7006, extra=[H1, H2, i])
    ctx = _ctx(N, s, d, C=C, K=K, K_ps=Kps, mode="column", split_rows=SPLIT)
    _say(f"huge rows, column mode: insert ({i}, {H1}), {len(block)} columns")
    ctx.apply_edge_update(i, H1, 1)
    got = ctx.query_columns(block).double().cpu().numpy().T
    ref = OI.delta_columns_c0(N, s.astype(np.int64), d.astype(np.int64), i, H1, block, C, K,
                              Kps)
    _say(f"  max |dS_gpu - dS_oracle| = {maxabs(got, ref):.3e}, max |dS| = "
         f"{np.abs(ref).max():.3e}")
    # same K and K_ps on both sides in float64; the output is rounded to float32
    assert np.all(np.abs(got - ref) <= 2.0 ** -24 * np.abs(ref) * 1.01 + 1e-13)
    ctx.close()


@pytest.mark.gpu
def test_huge_rows_fused_batch():
    s, d = _graph()
    into1 = _non_in_neighbours(s, d, H1, 20, seed=7007)
    into2 = _non_in_neighbours(s, d, H2, 3, seed=7008)
    g = W.rng(7009)
    bi, bj = list(into1) + list(into2), [H1] * 20 + [H2] * 3
    es = set(zip(s.tolist(), d.tolist()))
    while len(bi) < 40:
        x, y = (int(v) for v in g.integers(N, size=2))
        if x != y and (x, y) not in es and (x, y) not in zip(bi, bj):
            bi.append(x)
            bj.append(y)
    bo = [1] * len(bi)
    ctx = _ctx(N, s, d, C=C, K=25, s_prec="hilo", fused_batch=True, batch_chunk=8,
               split_rows=SPLIT)
    st = ctx.apply_batch(bi, bj, bo, stats=True)
    _say(f"huge rows, fused batch of {len(bi)} edges: {st['blocks']} blocks, "
         f"{st['fused_passes']} passes")
    tr = EdgeTracker(N, s, d)
    for x, y in zip(bi, bj):
        tr.apply(x, y, 1)
    cols = W.column_sample(N, 3, seed=7010, extra=[H1, H2, bi[0], bi[-1]])
    w = _check_columns(ctx, tr.Q(), cols, 1e-6)
    _say(f"  max |S_gpu - S*| over {len(cols)} columns = {w:.3e}")
    pairs = torch.as_tensor(np.stack([cols, cols[::-1]]), dtype=torch.int32)
    g1 = ctx.gather_pairs(pairs[0], pairs[1]).cpu().numpy()
    g2 = ctx.gather_pairs(pairs[1], pairs[0]).cpu().numpy()
    assert np.array_equal(g1, g2)
    ctx.close()
