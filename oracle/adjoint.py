"""Gradient of a pairwise squared loss on SimRank with respect to edge weights.

The paper has no gradient; this follows from eq (03a) by the chain rule. For a weighted
digraph, ``Q[x, y] = w(y -> x) / W_x`` with ``W_x`` the sum of x's in-edge weights. The loss
is ``L = sum_p (S[a_p, b_p] - t_p)^2`` over given pairs.

Differentiating eq (03a): ``dS = C (dQ S Q^T + Q S dQ^T) + C Q dS Q^T``, so
``dS = sum_k C^k Q^k [C (dQ S Q^T + Q S dQ^T)] (Q^T)^k``. With ``G = dL/dS`` (entries
``2 (S_ab - t)`` at (a, b)) and the adjoint ``Lam = sum_k C^k (Q^T)^k G Q^k``, the unique
solution of the transposed Sylvester equation ``Lam = G + C Q^T Lam Q``,

    dL/dQ = C (Lam + Lam^T) Q S                 (S symmetric)

and through the row normalisation ``dQ[x, y'] / dw(y -> x) = (delta_{y y'} - Q[x, y']) / W_x``,

    dL/dw(y -> x) = (dL/dQ[x, y] - sum_{y'} Q[x, y'] dL/dQ[x, y']) / W_x.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .graph import transition_matrix
from .simrank import depth_for, fixed_point, single_source


def loss(S, a, b, t):
    return float(np.sum((S[a, b] - t) ** 2))


def loss_grad_matrix(S, a, b, t):
    """G = dL/dS as a dense matrix (entries at (a_p, b_p) only)."""
    G = np.zeros_like(S)
    np.add.at(G, (a, b), 2.0 * (S[a, b] - t))
    return G


def adjoint_dense(Q, G, C, tol=1e-15, max_iter=400):
    """Iterate ``Lam <- G + C Q^T Lam Q`` from ``Lam = G`` to a step tolerance."""
    Qs = Q if sp.issparse(Q) else sp.csr_matrix(Q)
    QT = Qs.T.tocsr()
    L = G.copy()
    for _ in range(max_iter):
        P = np.asarray(QT @ L)                      # Q^T Lam
        Ln = G + C * np.asarray(QT @ P.T).T         # (Q^T (Q^T Lam)^T)^T = Q^T Lam Q
        step = float(np.max(np.abs(Ln - L)))
        L = Ln
        if step <= tol:
            break
    return L


def grad_weights_dense(n, src, dst, w, a, b, t, C, S=None, tol=1e-15):
    """dL/dw for every edge (edge order of ``src``/``dst``), dense; small n only."""
    Q = transition_matrix(n, src, dst, weight=w)
    if S is None:
        S = fixed_point(Q, C, tol=tol)
    G = loss_grad_matrix(S, a, b, t)
    Lam = adjoint_dense(Q, G, C, tol=tol)
    QS = np.asarray(Q @ S)
    dQ = C * (Lam + Lam.T) @ QS                     # dL/dQ, dense
    Qd = Q.toarray()
    rowterm = np.sum(Qd * dQ, axis=1)               # sum_y' Q[x,y'] dL/dQ[x,y']
    W = np.bincount(np.asarray(dst, dtype=np.int64), weights=np.asarray(w), minlength=n)
    x = np.asarray(dst, dtype=np.int64)
    y = np.asarray(src, dtype=np.int64)
    return (dQ[x, y] - rowterm[x]) / W[x], S, Lam


def lam_row(Q, QT, G, x, C, K):
    """Row x of ``Lam = sum_{k<=K} C^k (Q^T)^k G Q^k`` without forming Lam:
    ``Lam[x, :] = sum_k C^k r_k Q^k`` with ``r_k = (Q^k e_x)^T G``, summed by Horner's rule
    ``acc = r_K; acc = r_k + C acc Q`` (``acc Q`` computed as ``Q^T acc``)."""
    n = Q.shape[0]
    v = np.zeros(n)
    v[x] = 1.0
    rs = []
    for _k in range(K + 1):
        rs.append(np.asarray(G.T @ v).ravel())      # (v^T G)^T = G^T v
        v = Q @ v
    acc = rs[K]
    for k in range(K - 1, -1, -1):
        acc = rs[k] + C * (QT @ acc)
    return acc


def lam_col(Q, QT, G, x, C, K):
    """Column x of Lam: ``Lam[:, x] = sum_k C^k (Q^T)^k G Q^k e_x`` (Horner in Q^T)."""
    n = Q.shape[0]
    v = np.zeros(n)
    v[x] = 1.0
    cs = []
    for _k in range(K + 1):
        cs.append(np.asarray(G @ v).ravel())
        v = Q @ v
    acc = cs[K]
    for k in range(K - 1, -1, -1):
        acc = cs[k] + C * (QT @ acc)
    return acc


def grad_weight_edges(n, src, dst, w, a, b, t, C, edges, S_pairs=None, tol=1e-13,
                      g_pairs=None):
    """dL/dw for selected edge indices without dense matrices (large n).

    Needs S only at the loss pairs (``S_pairs``; computed by ``single_source`` when
    missing) and, per edge ``y -> x``, column y and column x of the converged S. Uses
    ``sum_{y'} Q[x, y'] (Q S)[:, y'] = (Q S Q^T)[:, x] = (S[:, x] - (1 - C) e_x) / C``.

    ``g_pairs``, when given, is dL/dS at the pairs directly (any upstream gradient, summed
    over repeated pairs); then ``t`` and ``S_pairs`` are not used.
    """
    Q = transition_matrix(n, src, dst, weight=w)
    QT = Q.T.tocsr()
    a = np.asarray(a, dtype=np.int64)
    b = np.asarray(b, dtype=np.int64)
    if g_pairs is None:
        if S_pairs is None:
            cache = {}
            S_pairs = np.empty(len(a))
            for p in range(len(a)):
                col = cache.get(int(b[p]))
                if col is None:
                    col = cache[int(b[p])] = single_source(Q, int(b[p]), C, tol)
                S_pairs[p] = col[a[p]]
        g_pairs = 2.0 * (S_pairs - t)
    G = sp.csr_matrix((np.asarray(g_pairs, dtype=np.float64), (a, b)), shape=(n, n))
    K = depth_for(C, tol)
    W = np.bincount(np.asarray(dst, dtype=np.int64), weights=np.asarray(w), minlength=n)
    out = np.empty(len(edges))
    for e_pos, e in enumerate(edges):
        x = int(dst[e])
        y = int(src[e])
        lam_x = lam_row(Q, QT, G, x, C, K) + lam_col(Q, QT, G, x, C, K)
        Sy = single_source(Q, y, C, tol)
        Sx = single_source(Q, x, C, tol)
        QSy = Q @ Sy
        dq_xy = C * float(lam_x @ QSy)
        ex = np.zeros(n)
        ex[x] = 1.0
        row = C * float(lam_x @ ((Sx - (1.0 - C) * ex) / C))
        out[e_pos] = (dq_xy - row) / W[x]
    return out


def fd_grad(n, src, dst, w, a, b, t, C, edges, h=1e-6, tol=1e-15):
    """Central finite differences of L (S recomputed to convergence) for selected edges."""
    out = np.empty(len(edges))
    for p, e in enumerate(edges):
        vals = []
        for s in (+1.0, -1.0):
            w2 = np.array(w, dtype=np.float64, copy=True)
            w2[e] += s * h
            Q = transition_matrix(n, src, dst, weight=w2)
            S = fixed_point(Q, C, tol=tol)
            vals.append(loss(S, a, b, t))
        out[p] = (vals[0] - vals[1]) / (2.0 * h)
    return out
