"""Incremental SimRank on a weighted digraph (test infrastructure: the oracle of the GPU
path, plain FP64 NumPy; only the tests and the benchmark's CPU leg use it).

The paper's updates are for unweighted graphs; this is their weighted analogue, derived the
same way. With row-normalised weights, ``Q[x, y] = w(y -> x) / W_x`` and ``W_x`` the sum of
x's in-edge weights. Changing the weight of one edge ``i -> j`` by ``dw`` (an insertion from
0, a deletion to 0, or a change of an existing edge's weight) moves row j of Q by a rank-one
term, the analogue of Theorem 1 (insertion) and Theorem 9 (deletion):

    Q'[j, :] = (W_j Q[j, :] + dw e_i) / (W_j + dw) = Q[j, :] + a (e_i - Q[j, :]),
    a = dw / (W_j + dw),

so ``Delta Q = u v^T`` with ``u = e_j``, ``v = a (e_i - Q[j, :])`` while ``W_j + dw > 0``;
removing j's last in-weight (``W_j + dw = 0``) gives ``v = -Q[j, :]``, and inserting into
an empty row (``W_j = 0``) gives ``v = e_i`` (both as in the unweighted theorems).

Theorem 2 then applies unchanged (it holds for any rank-one Delta Q). Theorem 3's closed
form carries over too, since its derivation uses only the fixed-point identity
``Q S Q^T = (S - (1 - C) I) / C`` (eq (33)), which the weighted Q satisfies as well:

    gamma = a (Q S e_i - S e_j / C) + (a (1 - C) / C + a^2 lambda / 2) e_j,
    lambda = S_ii + S_jj / C - 2 (Q S e_i)_j - 1/C + 1          (eq (29b), delta = 1).

With unit weights, ``a = 1 / (d_j + 1)`` for an insertion and ``-1 / (d_j - 1)`` for a
deletion, and the formulas are those of Theorems 1, 3 and 9.
"""
from __future__ import annotations

import numpy as np

from .incremental import gamma_from_direct, series


def rank_one_weight(Q, W, i, j, dw):
    """``Delta Q = u v^T`` for changing the weight of ``i -> j`` by ``dw`` (see above).
    ``Q`` dense (old), ``W`` old in-weight sums. Returns ``(u, v, a)``; ``a`` is None for
    the two cases without one (empty row before, or after)."""
    n = Q.shape[0]
    u = np.zeros(n)
    u[j] = 1.0
    Wn = W[j] + dw
    if W[j] == 0.0:                      # insertion into an empty row: Q'[j, :] = e_i
        v = np.zeros(n)
        v[i] = 1.0
        return u, v, None
    if Wn == 0.0:                        # the last in-weight removed: Q'[j, :] = 0
        return u, -np.asarray(Q[j, :], dtype=np.float64).copy(), None
    a = dw / Wn
    v = -a * np.asarray(Q[j, :], dtype=np.float64)
    v[i] += a
    return u, v, a


def gamma_closed_weight(QSi, Sj, Sii, j, C, a):
    """The closed form above from its ingredients ``QSi = Q S e_i``, ``Sj = S e_j``,
    ``Sii = S_ii`` and the scale ``a``."""
    lam = Sii + Sj[j] / C - 2.0 * QSi[j] - 1.0 / C + 1.0
    gamma = a * (QSi - Sj / C)
    gamma[j] += a * (1.0 - C) / C + 0.5 * a * a * lam
    return gamma


def inc_weight(Q, S, W, i, j, dw, C, K, form="closed"):
    """Delta of S for changing the weight of ``i -> j`` by ``dw`` on the weighted graph
    (dense ``Q``, ``S``, in-weight sums ``W``), by the series of eq (16a) to depth K.
    ``form="closed"``: the closed-form gamma (eq (29aa) for an empty row, Theorem 9's
    ``d_j = 1`` form when the last in-weight goes); ``form="direct"``: Theorem 2.
    Returns ``(S_new, info)``."""
    u, v, a = rank_one_weight(Q, W, i, j, dw)
    n = Q.shape[0]
    Si = S[:, i]
    QSi = Q @ Si
    if form == "direct":
        gamma = gamma_from_direct(Q, S, u, v, j)
    elif W[j] == 0.0:                    # eq (29aa)
        gamma = QSi.copy()
        gamma[j] += 0.5 * Si[i]
    elif W[j] + dw == 0.0:               # Theorem 9 with the last in-edge removed
        gamma = -QSi
        gamma[j] += 0.5 * Si[i]
    else:
        gamma = gamma_closed_weight(QSi, S[:, j], Si[i], j, C, a)
    xi0 = np.zeros(n)
    xi0[j] = C
    Xi, H = series(Q, u, v, xi0, gamma, C, K)
    M = Xi @ H.T
    return S + M + M.T, dict(u=u, v=v, a=a, gamma=gamma, Xi=Xi, H=H)
