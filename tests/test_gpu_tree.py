"""GPU parity of the forest-seeded all-pairs SimRank (Example 1.2) through the C ABI: the closed
form on a forest, the forest plus the other edges as one batch against the oracle's same
pipeline, and the rejections."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import graph as Gr
from oracle import incremental as OI
from oracle import simrank as O
from oracle import tree as T

from _util import maxabs

pytestmark = pytest.mark.gpu

C = 0.6


def _say(msg):
    print(msg, flush=True)


def ctx_for(n, s, d, **kw):
    from paper_1711_00121_amd import Context
    return Context(n, s, d, **kw)


def test_forest_closed_form_matches_oracle():
    """A graph that is its own spanning forest (several trees, no other edges): S is the
    closed form alone, every entry written by the kernel (n spans two column tiles and a
    ragged tail)."""
    n = 2100
    g = W.rng(801)
    parent = np.full(n, -1)
    for v in range(1, n):
        if g.random() > 0.01:                  # about 20 roots
            parent[v] = int(g.integers(max(0, v - 300), v))
    s = np.array([parent[v] for v in range(n) if parent[v] >= 0], dtype=np.int32)
    d = np.array([v for v in range(n) if parent[v] >= 0], dtype=np.int32)
    perm = g.permutation(len(s))
    s, d = s[perm], d[perm]
    _say(f"forest n={n}, {len(s)} edges")
    op, od = T.bfs_forest(n, s, d)
    ref = T.tree_simrank(op, od, C)
    ctx = ctx_for(n, s, d, init="forest", s_prec="fp64")
    assert ctx.init_stats["edges_in"] == 0
    S = ctx.S().cpu().numpy()
    assert maxabs(S, ref) < 1e-15
    assert np.count_nonzero(ref) < n * n // 4        # mostly zero across levels and trees
    ctx.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("hilo", 1e-6)])
def test_forest_seeded_matches_oracle(prec, tol):
    n, m = 300, 1500
    s, d = W.chung_lu(n, m, seed=811)
    _say(f"forest-seeded n={n} m={m} {prec}")
    ref = T.tree_seeded(n, s, d, C, 15)
    ctx = ctx_for(n, s, d, init="forest", s_prec=prec, K=15)
    S = ctx.S().cpu().numpy()
    st = ctx.init_stats
    parent, _ = T.bfs_forest(n, s, d)
    rest = ~T.tree_edges(n, s, d, parent)
    plan, _ = OI.plan_batch(n, s[~rest], d[~rest], s[rest], d[rest],
                            np.ones(rest.sum(), dtype=np.int64))
    assert st["edges_in"] == rest.sum() and st["blocks"] == len(plan)
    err = maxabs(S, ref)
    _say(f"max |S_gpu - S_oracle| = {err:.3e}")
    assert err < tol
    assert np.array_equal(S, S.T)
    # and the pipeline lands near the converged S of the whole graph
    exact = O.fixed_point(Gr.transition_matrix(n, s, d), C)
    assert maxabs(S, exact) < len(plan) * 2 * C ** 17 / (1 - C)
    ctx.close()


def test_forest_seeded_deep_series_reaches_fixed_point():
    """At K = 40 the seeded S equals the converged fixed point of eq (03a) to 1e-9 on a graph
    of several column tiles (n = 1500)."""
    n, m = 1500, 7500
    s, d = W.chung_lu(n, m, seed=821)
    _say(f"forest-seeded n={n} m={m} K=40")
    ctx = ctx_for(n, s, d, init="forest", s_prec="fp64", K=40)
    S = ctx.S().cpu().numpy()
    exact = O.fixed_point(Gr.transition_matrix(n, s, d), C)
    err = maxabs(S, exact)
    _say(f"max |S_gpu - S_exact| = {err:.3e}")
    assert err < 1e-9
    ctx.close()


def test_forest_seeded_rejections():
    from paper_1711_00121_amd._lib import SR_EMODE, SimRankError
    n = 50
    s, d = W.chung_lu(n, 200, seed=831)
    with pytest.raises(SimRankError) as e:
        ctx_for(n, s, d, init="forest", mode="column")
    assert e.value.status == SR_EMODE
    with pytest.raises(SimRankError):
        ctx_for(n, np.append(s, s[0]), np.append(d, d[0]), init="forest")   # duplicate
    with pytest.raises(SimRankError):
        ctx_for(n, np.append(s, 3), np.append(d, 3), init="forest")         # self-loop
    with pytest.raises(ValueError):
        ctx_for(n, s, d, init="forest", weight=np.ones(len(s)))
    torch.cuda.synchronize()


def test_forest_degenerate_graphs():
    """No edges: every node is a root and S = (1 - C) I; one node; a single path."""
    n = 1100
    ctx = ctx_for(n, np.zeros(0, np.int32), np.zeros(0, np.int32), init="forest",
                  s_prec="fp64")
    S = ctx.S().cpu().numpy()
    assert np.array_equal(S, (1.0 - C) * np.eye(n))
    ctx.close()
    one = ctx_for(1, np.zeros(0, np.int32), np.zeros(0, np.int32), init="forest")
    assert one.S().cpu().numpy().tolist() == [[1.0 - C]]
    one.close()
    n = 50                                     # a path 0 -> 1 -> ... -> 49 is its own tree
    s = np.arange(n - 1, dtype=np.int32)
    d = s + 1
    ctx = ctx_for(n, s, d, init="forest", s_prec="fp64")
    op, od = T.bfs_forest(n, s, d)
    assert maxabs(ctx.S().cpu().numpy(), T.tree_simrank(op, od, C)) < 1e-15
    ctx.close()
