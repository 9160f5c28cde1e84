"""GPU parity of all-pairs SimRank over a partitioned graph (Example 1.1) through the C ABI:
the block-by-block S against the oracle's, the blocks plus the cross-block batch against the
oracle's same pipeline, a deep series against the fixed point, and the rejections."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import graph as Gr
from oracle import incremental as OI
from oracle import partition as Pt
from oracle import simrank as O

from _util import maxabs

pytestmark = pytest.mark.gpu

C = 0.6


def _say(msg):
    print(msg, flush=True)


def ctx_for(n, s, d, **kw):
    from paper_1711_00121_amd import Context
    return Context(n, s, d, **kw)


def test_blocks_alone_match_oracle():
    """No cross-block edges: S is the block-diagonal S of the planted groups (n = 1500 over 6
    blocks of scattered ids)."""
    n = 1500
    s, d, g = W.communities(n, 7500, 6, 0.0, seed=951)
    _say(f"blocks alone n={n}")
    ctx = ctx_for(n, s, d, init="partitioned", part=g, s_prec="fp64")
    assert ctx.init_stats["edges_in"] == 0
    S = ctx.S().cpu().numpy()
    ref = Pt.block_simrank(n, s, d, g, C)
    err = maxabs(S, ref)
    _say(f"max |S_gpu - S_oracle| = {err:.3e}")
    assert err < 1e-13
    ctx.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("hilo", 1e-6)])
def test_partitioned_matches_oracle(prec, tol):
    n, m = 320, 1600
    s, d, _ = W.communities(n, m, 4, 0.05, seed=961)
    _say(f"partitioned n={n} m={m} {prec}")
    from paper_1711_00121_amd import partition
    lab = partition(n, s, d, 4)
    assert np.array_equal(lab, Pt.bfs_partition(n, s, d, 4))
    ref = Pt.partitioned(n, s, d, lab, C, 15)
    ctx = ctx_for(n, s, d, init="partitioned", parts=4, s_prec=prec, K=15)
    S = ctx.S().cpu().numpy()
    cross = lab[s] != lab[d]
    plan, _ = OI.plan_batch(n, s[~cross], d[~cross], s[cross], d[cross],
                            np.ones(cross.sum(), dtype=np.int64))
    st = ctx.init_stats
    assert st["edges_in"] == cross.sum() and st["blocks"] == len(plan)
    err = maxabs(S, ref)
    _say(f"max |S_gpu - S_oracle| = {err:.3e}")
    assert err < tol
    assert np.array_equal(S, S.T)
    ctx.close()


def test_partitioned_deep_series_reaches_fixed_point():
    n, m = 1200, 7200
    s, d, _ = W.communities(n, m, 8, 0.03, seed=971)
    _say(f"partitioned n={n} m={m} K=40")
    ctx = ctx_for(n, s, d, init="partitioned", parts=8, s_prec="fp64", K=40)
    S = ctx.S().cpu().numpy()
    exact = O.fixed_point(Gr.transition_matrix(n, s, d), C)
    err = maxabs(S, exact)
    _say(f"max |S_gpu - S_exact| = {err:.3e}")
    assert err < 1e-9
    ctx.close()


def test_partitioned_rejections():
    from paper_1711_00121_amd._lib import SR_EMODE, SR_ERANGE, SR_ESELF, SimRankError
    n = 60
    s, d, g = W.communities(n, 240, 3, 0.05, seed=981)
    with pytest.raises(SimRankError) as e:
        ctx_for(n, s, d, init="partitioned", part=g, mode="column")
    assert e.value.status == SR_EMODE
    bad = g.copy()
    bad[5] = n
    with pytest.raises(SimRankError) as e:
        ctx_for(n, s, d, init="partitioned", part=bad)
    assert e.value.status == SR_ERANGE
    with pytest.raises(SimRankError) as e:
        ctx_for(n, np.append(s, 4), np.append(d, 4), init="partitioned", part=g)
    assert e.value.status == SR_ESELF
    with pytest.raises(ValueError):
        ctx_for(n, s, d, init="partitioned", part=g[:-1])
    torch.cuda.synchronize()


def test_partition_extremes():
    """One block (no cross edges): the fixed point of the whole graph. Singleton blocks (every
    edge crosses): the oracle's pipeline from S = (1 - C) I."""
    n, m = 240, 1000
    s, d, _ = W.communities(n, m, 3, 0.05, seed=991)
    one = ctx_for(n, s, d, init="partitioned", parts=1, s_prec="fp64")
    assert one.init_stats["edges_in"] == 0
    exact = O.fixed_point(Gr.transition_matrix(n, s, d), C)
    assert maxabs(one.S().cpu().numpy(), exact) < 1e-13
    one.close()
    lab = np.arange(n)
    ref = Pt.partitioned(n, s, d, lab, C, 15)
    sing = ctx_for(n, s, d, init="partitioned", part=lab, s_prec="fp64", K=15)
    assert sing.init_stats["edges_in"] == m
    assert maxabs(sing.S().cpu().numpy(), ref) < 1e-12
    sing.close()
