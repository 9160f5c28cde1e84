"""Pins of the oracle's edge-weight gradient: central finite differences of the recomputed
loss, the incremental Delta S of a weight perturbation (a rank-one Delta Q, the weighted
form of Theorem 1) taken as a directional derivative, the scale invariance of each row of Q
(Euler's identity), and the per-edge large-graph form against the dense form."""
import numpy as np

from oracle import adjoint as A
from oracle import graph as Gr
from oracle import incremental as I
from oracle import simrank as O

C = 0.6


def weighted_graph(seed, n=9, p=0.35):
    rng = np.random.default_rng(seed)
    e = [(a, b) for a in range(n) for b in range(n) if a != b and rng.random() < p]
    s = np.array([a for a, _ in e], dtype=np.int64)
    d = np.array([b for _, b in e], dtype=np.int64)
    w = np.exp(rng.normal(0.0, 0.5, len(e)))
    a = np.array([0, 1, 2, 3, 1])
    b = np.array([4, 5, 6, 7, 8])
    t = rng.uniform(0.0, 0.2, len(a))
    return n, s, d, w, a, b, t


def test_gradient_matches_central_differences():
    for seed in (0, 1):
        n, s, d, w, a, b, t = weighted_graph(seed)
        g, S, _ = A.grad_weights_dense(n, s, d, w, a, b, t, C)
        fd = A.fd_grad(n, s, d, w, a, b, t, C, list(range(len(s))), h=1e-6)
        assert np.abs(g - fd).max() < 1e-9 * max(1.0, np.abs(g).max())


def test_euler_identity_and_single_in_edge():
    # Q's row x is invariant under scaling all of x's in-edge weights, so
    # sum_y w(y->x) dL/dw(y->x) = 0; a node with one in-edge has gradient 0 on it.
    n, s, d, w, a, b, t = weighted_graph(3, n=10, p=0.3)
    g, _, _ = A.grad_weights_dense(n, s, d, w, a, b, t, C)
    for x in range(n):
        sel = d == x
        if sel.any():
            assert abs(np.sum(w[sel] * g[sel])) < 1e-15
        if sel.sum() == 1:
            assert abs(g[sel][0]) < 1e-15


def test_directional_derivative_from_incremental_update():
    """Perturbing w(y -> x) by eps changes row x of Q by the rank-one
    (eps / (W_x + eps)) e_x (e_y - Q[x, :])^T. The first-order part of the incremental
    Delta S (w = Q S v, no lambda u u^T term, Q in place of Q~) is eps * dS/dw, so
    <G, that part> / eps equals dL/dw."""
    n, s, d, w, a, b, t = weighted_graph(4)
    Q = Gr.transition_matrix(n, s, d, weight=w, dense=True)
    S = O.fixed_point(Gr.transition_matrix(n, s, d, weight=w), C)
    G = A.loss_grad_matrix(S, a, b, t)
    g, _, _ = A.grad_weights_dense(n, s, d, w, a, b, t, C)
    W = np.bincount(d, weights=w, minlength=n)
    for e in range(0, len(s), 3):
        x, y = int(d[e]), int(s[e])
        ex = np.eye(n)[x]
        v = np.eye(n)[y] - Q[x, :]
        u = ex / W[x]                                  # derivative of eps/(W_x+eps) at 0
        y_vec = Q @ (S @ v)
        zero = np.zeros(n)
        Xi, H = I.series(Q, zero, zero, C * u, y_vec, C, 90)
        M = Xi @ H.T
        dS = M + M.T
        assert abs(np.sum(G * dS) - g[e]) < 1e-12
        # and the full incremental update is consistent at second order
        eps = 1e-4
        u_eps = ex * eps / (W[x] + eps)
        ws = I.w_direct(Q, S, u_eps, v)
        Xi, H = I.series(Q, u_eps, v, C * u_eps, ws, C, 90)
        M = Xi @ H.T
        w2 = w.copy()
        w2[e] += eps
        S2 = O.fixed_point(Gr.transition_matrix(n, s, d, weight=w2), C)
        assert np.abs(S + M + M.T - S2).max() < 1e-13


def test_edge_form_equals_dense_form():
    n, s, d, w, a, b, t = weighted_graph(5, n=11, p=0.3)
    g, S, _ = A.grad_weights_dense(n, s, d, w, a, b, t, C)
    ge = A.grad_weight_edges(n, s, d, w, a, b, t, C, list(range(len(s))))
    assert np.abs(ge - g).max() < 1e-13


def test_edge_form_with_upstream_gradient():
    """Any upstream dL/dS at the pairs: the edge form equals the dense chain rule taken with
    that G (pins the g_pairs path used at large n), and a repeated pair adds up."""
    n, s, d, w, a, b, t = weighted_graph(7, n=11, p=0.3)
    a = np.concatenate([a, a[:2]])
    b = np.concatenate([b, b[:2]])
    rng = np.random.default_rng(8)
    gp = rng.normal(size=len(a))
    Q = Gr.transition_matrix(n, s, d, weight=w)
    S = O.fixed_point(Q, C)
    G = np.zeros((n, n))
    np.add.at(G, (a, b), gp)
    Lam = A.adjoint_dense(Q, G, C)
    dQ = C * (Lam + Lam.T) @ np.asarray(Q @ S)
    Qd = Q.toarray()
    Wx = np.bincount(d, weights=w, minlength=n)
    ref = (dQ[d, s] - np.sum(Qd * dQ, axis=1)[d]) / Wx[d]
    ge = A.grad_weight_edges(n, s, d, w, a, b, None, C, list(range(len(s))), g_pairs=gp)
    assert np.abs(ge - ref).max() < 1e-13 * max(1.0, np.abs(ref).max())
    # central differences of the linear functional sum_p gp S[a_p, b_p]
    for e in (0, len(s) // 2, len(s) - 1):
        vals = []
        for sg in (1.0, -1.0):
            w2 = w.copy()
            w2[e] += sg * 1e-6
            S2 = O.fixed_point(Gr.transition_matrix(n, s, d, weight=w2), C)
            vals.append(float(np.sum(gp * S2[a, b])))
        assert abs((vals[0] - vals[1]) / 2e-6 - ge[e]) < 1e-8


def test_adjoint_solves_transposed_sylvester():
    n, s, d, w, a, b, t = weighted_graph(6)
    Q = Gr.transition_matrix(n, s, d, weight=w, dense=True)
    S = O.fixed_point(Gr.transition_matrix(n, s, d, weight=w), C)
    G = A.loss_grad_matrix(S, a, b, t)
    L = A.adjoint_dense(Q, G, C)
    assert np.abs(G + C * Q.T @ L @ Q - L).max() < 1e-15
