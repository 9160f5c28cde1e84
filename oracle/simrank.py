"""SimRank matrix S of Li et al.'s model (section 3.1, eq (03a)):

    S = C * Q * S * Q^T + (1 - C) * I_n,    0 < C < 1.

Because C < 1 and every row of Q sums to 1 or 0, the map is a contraction in the max-norm
and S is its unique fixed point; the series form is eq (17):
``S = (1 - C) * sum_k C^k Q^k (Q^T)^k``.

Functions:

* ``kron_solve``    exact solve through the Kronecker (vec) form of eq (03a); tiny n only.
* ``fixed_point``   the iteration ``S <- C Q S Q^T + (1 - C) I`` to a step tolerance.
* ``partial_sim``   the PartialSim procedure of section 7 (one column from K steps).
* ``single_source`` one column of the converged S, by PartialSim run deep enough that the
                    dropped tail ``C^(K+1)`` is below a tolerance.
* ``truncated``     the K-term partial sum of eq (17), dense (for pins of PartialSim).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp


def _dense(Q):
    return Q.toarray() if sp.issparse(Q) else np.asarray(Q, dtype=np.float64)


def kron_solve(Q, C):
    """vec(S) = (1 - C) (I - C Q kron Q)^{-1} vec(I), from vec(A X B) = (B^T kron A) vec(X)
    applied to eq (03a). O(n^6): n <= 12 only."""
    Qd = _dense(Q)
    n = Qd.shape[0]
    if n > 12:
        raise ValueError("kron_solve is for tiny graphs")
    A = np.eye(n * n) - C * np.kron(Qd, Qd)
    s = np.linalg.solve(A, (1.0 - C) * np.eye(n).reshape(-1))
    return s.reshape(n, n)


def fixed_point(Q, C, tol=1e-15, S0=None, max_iter=400, return_iters=False):
    """Iterate ``S_{t+1} = C Q S_t Q^T + (1 - C) I`` from ``S0`` (default ``(1 - C) I``)
    until ``max |S_{t+1} - S_t| <= tol``.

    The remaining error is at most ``C / (1 - C) * tol`` (contraction factor C). When
    rounding keeps the step above ``tol``, the iteration stops once the step no longer
    decreases over 5 consecutive iterations.
    """
    n = Q.shape[0]
    Qs = Q if sp.issparse(Q) else sp.csr_matrix(Q)
    S = (1.0 - C) * np.eye(n) if S0 is None else np.array(S0, dtype=np.float64, copy=True)
    best = math.inf
    stall = 0
    it = 0
    for it in range(1, max_iter + 1):
        P = np.asarray(Qs @ S)                       # Q S
        S_new = C * np.asarray(Qs @ P.T).T          # (Q (Q S)^T)^T = Q S Q^T
        S_new[np.diag_indices(n)] += 1.0 - C
        step = float(np.max(np.abs(S_new - S))) if n else 0.0
        S = S_new
        if step <= tol:
            break
        if step < best:
            best = step
            stall = 0
        else:
            stall += 1
            if stall >= 5:
                break
    return (S, it) if return_iters else S


def truncated(Q, C, K):
    """``S_K = (1 - C) sum_{k=0}^{K} C^k Q^k (Q^T)^k`` (eq (17) cut after K+1 terms),
    which is also the K-th fixed-point iterate started from ``(1 - C) I``."""
    Qd = _dense(Q)
    n = Qd.shape[0]
    S = np.zeros((n, n))
    Qk = np.eye(n)
    for k in range(K + 1):
        S += (C ** k) * (Qk @ Qk.T)
        Qk = Qd @ Qk
    return (1.0 - C) * S


def partial_sim(Q, q, K, C):
    """PartialSim (section 7, Procedure PartialSim): column q of the K-term SimRank.

    The printed procedure starts from ``x_0 = e_q`` but its loop builds ``x_{t+1}`` from
    ``x_t`` for t = 1..K, which leaves ``x_1`` undefined. Reading used here:
    ``x_0 = e_q``; ``x_t = Q^T x_{t-1}`` for t = 1..K; ``y = x_K``; then for t = 1..K,
    ``y = x_{K-t} + C Q y``; return ``(1 - C) y``. This equals column q of ``truncated``.
    """
    n = Q.shape[0]
    Qs = Q if sp.issparse(Q) else sp.csr_matrix(Q)
    QT = Qs.T.tocsr()
    xs = [np.zeros(n)]
    xs[0][q] = 1.0
    for t in range(1, K + 1):
        xs.append(QT @ xs[t - 1])
    y = xs[K].copy()
    for t in range(1, K + 1):
        y = xs[K - t] + C * (Qs @ y)
    return (1.0 - C) * y


def depth_for(C, tol):
    """Smallest K with C^(K+1) <= tol: the tail of eq (17) past K is below tol entrywise."""
    return max(1, int(math.ceil(math.log(tol) / math.log(C))) - 1)


def single_source(Q, q, C, tol=1e-14):
    """Column q of the converged S to within ``tol`` (max-abs).

    Each term ``C^k Q^k (Q^T)^k e_q`` of eq (17) has entries in [0, C^k] because
    ``||(Q^T)^k e_q||_1 <= 1`` and Q^k does not increase the max-norm, so the tail after K
    terms is at most ``(1 - C) sum_{k>K} C^k = C^(K+1)``.
    """
    return partial_sim(Q, q, depth_for(C, tol), C)
