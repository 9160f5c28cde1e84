"""Weighted graphs on the GPU through the C ABI: unit updates of every kind (insertion into a
filled and an empty row, weight up and down, deletion with in-edges left and of the last one,
new sink, new source, two new nodes) against the oracle's weighted updates at the same K
(1e-12) and the converged recompute (1e-6); the incremental Delta S of a small weight change
taken as a directional derivative against the adjoint's dL/dw; and dL/dw after updates
against the oracle's gradient of the updated graph."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import adjoint as A
from oracle import graph as Gr
from oracle import simrank as O
from oracle import weighted as Wt

from _util import maxabs

pytestmark = pytest.mark.gpu

C = 0.6


def ctx_for(n, s, d, w, **kw):
    from paper_1711_00121_amd import Context
    return Context(n, s, d, weight=w, **kw)


class WeightedTracker:
    """Weighted edge list (oracle side), updated alongside the GPU context."""

    def __init__(self, n, s, d, w):
        self.n = n
        self.es = {(a, b): x for a, b, x in zip(s.tolist(), d.tolist(), w.tolist())}

    def arrays(self):
        k = sorted(self.es)
        return (np.array([a for a, _ in k], dtype=np.int64),
                np.array([b for _, b in k], dtype=np.int64), np.array([self.es[x] for x in k]))

    def dense(self, nn=None):
        nn = self.n if nn is None else nn
        s, d, w = self.arrays()
        Q = np.zeros((nn, nn))
        Q[:self.n, :self.n] = Gr.transition_matrix(self.n, s, d, weight=w, dense=True)
        Wsum = np.zeros(nn)
        Wsum[:self.n] = np.bincount(d, weights=w, minlength=self.n)
        return Q, Wsum

    def exact(self):
        s, d, w = self.arrays()
        return O.fixed_point(Gr.transition_matrix(self.n, s, d, weight=w), C)

    def set(self, i, j, x):
        if x == 0.0:
            del self.es[(i, j)]
        else:
            self.es[(i, j)] = x
        self.n = max(self.n, i + 1, j + 1)


def update_sequence(n, s, d, w):
    es = {(a, b): x for a, b, x in zip(s.tolist(), d.tolist(), w.tolist())}
    indeg = np.bincount(d, minlength=n)
    hub = int(np.argmax(indeg))
    free = next(a for a in range(n) if a != hub and (a, hub) not in es)
    empty = next(x for x in range(n) if indeg[x] == 0)
    multi = next(e for e in sorted(es) if indeg[e[1]] >= 3 and e[1] != hub)
    single = next(e for e in sorted(es) if indeg[e[1]] == 1)
    e0 = sorted(es)[11]
    return [
        (free, hub, 1.7),                        # insertion into a filled row
        (3 if empty != 3 else 4, empty, 0.45),   # insertion into an empty row
        (e0[0], e0[1], es[e0] * 2.5),            # weight up
        (e0[0], e0[1], es[e0] * 0.3),            # weight down
        (multi[0], multi[1], 0.0),               # deletion, other in-edges left
        (single[0], single[1], 0.0),             # deletion of the last in-edge
        (5, n, 0.9),                             # new sink (C1)
        (n + 1, hub, 1.3),                       # new source (C2)
        (n + 2, n + 3, 0.7),                     # two new nodes (C3)
    ]


def test_weighted_unit_updates_match_oracle():
    n = 300
    s, d = W.chung_lu(n, 1800, seed=971)
    w = W.lognormal_weights(len(s), seed=972)
    K = 15
    ctx = ctx_for(n, s, d, w, C=C, K=K, s_prec="fp64", node_cap=n + 8)
    deep = ctx_for(n, s, d, w, C=C, K=45, s_prec="fp64", node_cap=n + 8)
    tr = WeightedTracker(n, s, d, w)
    S_or = tr.exact()
    assert maxabs(ctx.S().cpu().numpy(), S_or) < 1e-13
    for (i, j, x) in update_sequence(n, s, d, w):
        nn = max(tr.n, i + 1, j + 1)
        Q, Wsum = tr.dense(nn)
        G = np.zeros((nn, nn))
        G[:tr.n, :tr.n] = S_or
        for t in range(tr.n, nn):
            G[t, t] = 1.0 - C
        w_old = tr.es.get((i, j), 0.0)
        S_or, _ = Wt.inc_weight(Q, G, Wsum, i, j, x - w_old, C, K)
        st = ctx.apply_weight_update(i, j, x, stats=True)
        deep.apply_weight_update(i, j, x)
        tr.set(i, j, x)
        assert ctx.sizes() == (tr.n, len(tr.es)) and st["n_after"] == tr.n
        S = ctx.S().cpu().numpy()
        assert maxabs(S, S_or) < 1e-12, (i, j, w_old, x, maxabs(S, S_or))
        assert maxabs(deep.S().cpu().numpy(), tr.exact()) < 1e-6, (i, j, w_old, x)
        src, dst, ww = ctx.edges()
        assert sorted(zip(src.tolist(), dst.tolist(), ww.tolist())) == \
            sorted((a, b, v) for (a, b), v in tr.es.items())
    # apply_edge_update on a weighted graph: an insertion of weight 1 and a deletion
    es = tr.es
    i, j = next((a, b) for a in range(tr.n) for b in range(40) if a != b and (a, b) not in es)
    ctx.apply_edge_update(i, j, 1)
    tr.set(i, j, 1.0)
    e = sorted(es)[5]
    ctx.apply_edge_update(e[0], e[1], -1)
    tr.set(e[0], e[1], 0.0)
    assert maxabs(ctx.S().cpu().numpy(), tr.exact()) < 1e-6
    ctx.close()
    deep.close()


def test_weight_change_rejections():
    from paper_1711_00121_amd import _lib as L
    n = 60
    s, d = W.chung_lu(n, 200, seed=973)
    w = W.lognormal_weights(len(s), seed=974)
    ctx = ctx_for(n, s, d, w, C=C, K=8, s_prec="fp64", node_cap=n + 2)
    S0 = ctx.S().cpu().numpy()
    es = set(zip(s.tolist(), d.tolist()))
    free = next((a, b) for a in range(n) for b in range(n) if a != b and (a, b) not in es)

    def status(*a):
        try:
            ctx.apply_weight_update(*a)
        except L.SimRankError as e:
            return e.status
        return L.SR_OK

    assert status(free[0], free[1], 0.0) == L.SR_ENOENT
    assert status(int(s[0]), int(d[0]), -1.0) == L.SR_EINVAL
    assert status(int(s[0]), int(d[0]), float("nan")) == L.SR_EINVAL
    assert status(4, 4, 1.0) == L.SR_ESELF
    assert status(3, n + 1, 1.0) == L.SR_ERANGE
    assert status(int(s[0]), int(d[0]), float(w[0])) == L.SR_OK   # unchanged: no update
    assert np.array_equal(ctx.S().cpu().numpy(), S0)
    from paper_1711_00121_amd import Context
    plain = Context(n, s, d, C=C, K=8, s_prec="fp64")
    with pytest.raises(L.SimRankError) as ei:
        plain.apply_weight_update(int(s[0]), int(d[0]), 2.0)
    assert ei.value.status == L.SR_EMODE
    plain.close()
    ctx.close()


def test_incremental_delta_is_the_directional_derivative():
    """For L = sum_p g_p S[a_p, b_p], the incremental Delta S of a small weight change
    (w_e -> w_e + eps) contracted with g and divided by eps is dL/dw_e of the adjoint."""
    n = 500
    s, d = W.chung_lu(n, 3000, seed=975)
    w = W.lognormal_weights(len(s), seed=976)
    ctx = ctx_for(n, s, d, w, C=C, K=40, s_prec="fp64")
    a, b, t = W.loss_pairs(n, 64, seed=977)
    at = torch.as_tensor(a, dtype=torch.int32, device="cuda")
    bt = torch.as_tensor(b, dtype=torch.int32, device="cuda")
    g = 2.0 * (ctx.gather_pairs(at, bt) - torch.as_tensor(t, device="cuda"))
    dw = ctx.backward(at, bt, g).cpu().numpy()
    gh = g.cpu().numpy()
    src, dst, ww = ctx.edges()
    indeg = np.bincount(dst, minlength=n)
    picks = [e for e in range(0, len(src), 97) if indeg[dst[e]] >= 2][:8]
    worst = 0.0
    for e in picks:
        i, j, x = int(src[e]), int(dst[e]), float(ww[e])
        eps = 1e-5 * x
        v0 = ctx.gather_pairs(at, bt).cpu().numpy()
        ctx.apply_weight_update(i, j, x + eps)
        v1 = ctx.gather_pairs(at, bt).cpu().numpy()
        ctx.apply_weight_update(i, j, x)
        dd = float(np.sum(gh * (v1 - v0))) / eps
        rel = abs(dd - dw[e]) / max(abs(dw[e]), 1e-3 * np.abs(dw).max())
        worst = max(worst, rel)
        assert rel < 1e-4, (e, dd, dw[e])
    print(f"directional derivative vs adjoint: worst relative difference {worst:.2e}")
    ctx.close()


@pytest.mark.parametrize("weighted", [True, False])
def test_backward_after_updates(weighted):
    """dL/dw after updates (the stored S is the incrementally maintained one) against the
    oracle's gradient of the updated graph, in the order of Context.edges."""
    n = 240
    s, d = W.chung_lu(n, 1400, seed=978)
    w = W.lognormal_weights(len(s), seed=979) if weighted else None
    from paper_1711_00121_amd import Context
    ctx = Context(n, s, d, weight=w, C=C, K=40, s_prec="fp64", node_cap=n + 4)
    es = set(zip(s.tolist(), d.tolist()))
    free = [(x, y) for x in range(n) for y in range(0, n, 7) if x != y and (x, y) not in es]
    dele = sorted(es)[::211][:3]
    if weighted:
        ctx.apply_weight_update(*free[0], 1.4)
        ctx.apply_weight_update(*free[1], 0.6)
        ctx.apply_weight_update(dele[0][0], dele[0][1], 0.0)
        ctx.apply_weight_update(dele[1][0], dele[1][1], 2.2)
        ctx.apply_weight_update(3, n, 0.8)
        ctx.apply_weight_update(n + 1, 9, 1.1)
    else:
        ctx.apply_edge_update(*free[0], 1)
        ctx.apply_edge_update(*free[1], 1)
        ctx.apply_edge_update(dele[0][0], dele[0][1], -1)
        ctx.apply_edge_update(3, n, 1)
        ctx.apply_edge_update(n + 1, 9, 1)
    n2, m2 = ctx.sizes()
    src, dst, ww = ctx.edges()
    assert len(src) == m2
    a, b, t = W.loss_pairs(n2, 48, seed=980)
    g_or, S_or, _ = A.grad_weights_dense(n2, src.astype(np.int64), dst.astype(np.int64), ww,
                                         a, b, t, C)
    at = torch.as_tensor(a, dtype=torch.int32, device="cuda")
    bt = torch.as_tensor(b, dtype=torch.int32, device="cuda")
    gp = 2.0 * (torch.as_tensor(S_or[a, b], device="cuda") - torch.as_tensor(t, device="cuda"))
    got = ctx.backward(at, bt, gp).cpu().numpy()
    err = np.abs(got - g_or).max() / np.abs(g_or).max()
    print(f"backward after updates ({'weighted' if weighted else 'unweighted'}): "
          f"relative max difference {err:.2e}")
    assert err < 1e-8
    # SimRankPairs checks the weights against the updated context's
    from paper_1711_00121_amd import simrank_pairs
    wt = torch.tensor(ww, dtype=torch.float64, device="cuda", requires_grad=True)
    v = simrank_pairs(wt, ctx, at, bt)
    (gp * v).sum().backward()
    assert np.abs(wt.grad.cpu().numpy() - g_or).max() / np.abs(g_or).max() < 1e-8
    ctx.close()
