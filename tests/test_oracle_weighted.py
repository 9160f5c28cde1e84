"""Pins of the oracle's weighted updates (the weighted analogue of Theorems 1-3 and 9):
the rank-one term reproduces the recomputed transition matrix exactly; the closed and the
direct forms agree; both reach the recompute of the updated weighted graph; unit weights
reduce to the unweighted updates; node insertions work as isolated nodes plus an update; and
a small weight change divided by itself is the gradient of the adjoint."""
import numpy as np
import pytest

from oracle import adjoint as A
from oracle import graph as Gr
from oracle import incremental as I
from oracle import simrank as O
from oracle import weighted as Wt

C = 0.6


def graph(seed, n=10, p=0.3):
    rng = np.random.default_rng(seed)
    e = [(a, b) for a in range(n) for b in range(n) if a != b and rng.random() < p]
    s = np.array([a for a, _ in e], dtype=np.int64)
    d = np.array([b for _, b in e], dtype=np.int64)
    w = np.exp(rng.normal(0.0, 0.5, len(e)))
    return n, s, d, w


def state(n, s, d, w):
    Q = Gr.transition_matrix(n, s, d, weight=w, dense=True)
    W = np.bincount(d, weights=w, minlength=n).astype(np.float64)
    return Q, W, O.kron_solve(Q, C)


def changed(n, s, d, w, i, j, w_new):
    """Edge list with the weight of i -> j set to w_new (0 removes it)."""
    es = {(a, b): x for a, b, x in zip(s.tolist(), d.tolist(), w.tolist())}
    if w_new == 0.0:
        del es[(i, j)]
    else:
        es[(i, j)] = w_new
    k = sorted(es)
    return (np.array([a for a, _ in k], dtype=np.int64), np.array([b for _, b in k], dtype=np.int64),
            np.array([es[x] for x in k]))


def cases(n, s, d, w):
    """(i, j, w_old, w_new): insertion into a non-empty and into an empty row, deletion with
    other in-edges left and of a sink's last in-edge, weight up and down."""
    es = {(a, b): x for a, b, x in zip(s.tolist(), d.tolist(), w.tolist())}
    indeg = np.bincount(d, minlength=n)
    out = []
    j = int(np.argmax(indeg))
    i = next(a for a in range(n) if a != j and (a, j) not in es)
    out.append((i, j, 0.0, 1.7))
    empty = [x for x in range(n) if indeg[x] == 0]
    if empty:
        out.append((0 if empty[0] != 0 else 1, empty[0], 0.0, 0.4))
    multi = next(((a, b) for (a, b) in es if indeg[b] >= 2), None)
    out.append((multi[0], multi[1], es[multi], 0.0))
    single = next(((a, b) for (a, b) in es if indeg[b] == 1), None)
    if single:
        out.append((single[0], single[1], es[single], 0.0))
    e0 = sorted(es)[3]
    out.append((e0[0], e0[1], es[e0], es[e0] * 2.5))
    out.append((e0[0], e0[1], es[e0], es[e0] * 0.3))
    return out


def test_rank_one_term_reproduces_the_new_transition_matrix():
    for seed in (1, 2, 3):
        n, s, d, w = graph(seed)
        Q, W, _ = state(n, s, d, w)
        for i, j, w_old, w_new in cases(n, s, d, w):
            u, v, _ = Wt.rank_one_weight(Q, W, i, j, w_new - w_old)
            s2, d2, w2 = changed(n, s, d, w, i, j, w_new)
            Q2 = Gr.transition_matrix(n, s2, d2, weight=w2, dense=True)
            assert np.abs(Q + np.outer(u, v) - Q2).max() < 1e-15, (seed, i, j, w_old, w_new)


def test_closed_and_direct_forms_reach_the_recompute():
    for seed in (4, 5):
        n, s, d, w = graph(seed)
        Q, W, S = state(n, s, d, w)
        for i, j, w_old, w_new in cases(n, s, d, w):
            s2, d2, w2 = changed(n, s, d, w, i, j, w_new)
            exact = O.kron_solve(Gr.transition_matrix(n, s2, d2, weight=w2, dense=True), C)
            Sc, _ = Wt.inc_weight(Q, S, W, i, j, w_new - w_old, C, 80, "closed")
            Sd, _ = Wt.inc_weight(Q, S, W, i, j, w_new - w_old, C, 80, "direct")
            assert np.abs(Sc - exact).max() < 1e-12, (seed, i, j, w_old, w_new)
            assert np.abs(Sd - exact).max() < 1e-12
            # at a short series the two forms still agree (S is an exact fixed point here)
            Sc5, _ = Wt.inc_weight(Q, S, W, i, j, w_new - w_old, C, 5, "closed")
            Sd5, _ = Wt.inc_weight(Q, S, W, i, j, w_new - w_old, C, 5, "direct")
            assert np.abs(Sc5 - Sd5).max() < 1e-13


def test_unit_weights_reduce_to_the_unweighted_updates():
    n, s, d, _ = graph(6)
    w = np.ones(len(s))
    Q, W, S = state(n, s, d, w)
    dg = np.bincount(d, minlength=n)
    for i, j, w_old, w_new in cases(n, s, d, w):
        if w_old not in (0.0, 1.0) or w_new not in (0.0, 1.0):
            continue
        op = 1 if w_new > w_old else -1
        Sw, info = Wt.inc_weight(Q, S, W, i, j, w_new - w_old, C, 12)
        Su, iu = I.inc_usr(Q, S, dg, i, j, C, 12, op=op)
        assert np.abs(Sw - Su).max() < 1e-14
        assert np.abs(np.outer(info["u"], info["v"]) - np.outer(iu["u"], iu["v"])).max() < 1e-15


def test_node_insertions_as_isolated_nodes_then_an_update():
    """C1 (new sink), C2 (new source) and C3 (both new) with weights: grow S by isolated
    nodes (diagonal 1 - C), then the weighted insertion; equal to the recompute."""
    n, s, d, w = graph(7)
    es_w = list(zip(s.tolist(), d.tolist(), w.tolist()))
    for (i, j, nn) in [(2, n, n + 1), (n, 3, n + 1), (n, n + 1, n + 2)]:
        Q, W, S = state(n, s, d, w)
        G = np.zeros((nn, nn))
        G[:n, :n] = S
        for x in range(n, nn):
            G[x, x] = 1.0 - C
        Qg = np.zeros((nn, nn))
        Qg[:n, :n] = Q
        Wg = np.concatenate([W, np.zeros(nn - n)])
        S2, _ = Wt.inc_weight(Qg, G, Wg, i, j, 0.8, C, 60)
        s2 = np.array([a for a, _, _ in es_w] + [i], dtype=np.int64)
        d2 = np.array([b for _, b, _ in es_w] + [j], dtype=np.int64)
        w2 = np.array([x for _, _, x in es_w] + [0.8])
        exact = O.kron_solve(Gr.transition_matrix(nn, s2, d2, weight=w2, dense=True), C)
        assert np.abs(S2 - exact).max() < 1e-12, (i, j)


def test_small_weight_change_is_the_adjoint_gradient():
    """(S(w + eps e_e) - S(w)) / eps by the incremental update, contracted with dL/dS, is
    dL/dw_e of the adjoint to first order in eps."""
    n, s, d, w = graph(8)
    Q, W, S = state(n, s, d, w)
    a = np.array([0, 1, 2, 5])
    b = np.array([3, 4, 6, 9])
    t = np.array([0.05, 0.1, 0.0, 0.2])
    g, _, _ = A.grad_weights_dense(n, s, d, w, a, b, t, C)
    G = A.loss_grad_matrix(S, a, b, t)
    for e in range(0, len(s), 4):
        eps = 1e-7 * w[e]
        S2, _ = Wt.inc_weight(Q, S, W, int(s[e]), int(d[e]), eps, C, 80)
        fd = float(np.sum(G * (S2 - S))) / eps
        assert abs(fd - g[e]) < 1e-6 * max(1.0, abs(g[e])), (e, fd, g[e])
