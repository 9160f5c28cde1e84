"""Dense FP64 evaluations of the paper's incremental SimRank formulas, in the paper's order
and notation. These are slow (dense n x n) and meant for small graphs: they pin the
incremental method against recomputation, and they give reference intermediate quantities
(u, v, gamma, the series vectors, affected-area sets, batch plans).

Notation: ``Q`` old backward transition matrix (dense), ``S`` old SimRank matrix, ``d``
integer in-degrees of the old graph, edge ``(i, j)`` means ``i -> j`` (j is the sink whose
row of Q changes), ``C`` damping, ``K`` number of iterations (K + 1 series terms,
k = 0..K, as Algorithm 1 sets M_0 and then runs K updates).

Readings taken where the paper is silent or garbled (each one listed in the design notes):

* Table 2 deletion conditions "(d_j = 1) / (d_j > 1)" are read as (d_j = delta) /
  (d_j > delta); only deleting all of j's in-edges empties row j.
* Table 2's indicator ``e_I`` is 1 on I and 0 elsewhere; ``S[:, I]`` is the sum of the
  columns in I and ``S_{I,I} = e_I^T S e_I``.
* Affected areas (Theorem 4) use the product of projections, propagated structurally by
  out-neighbour search; the final update covers the union rectangle
  ``A_hat x B_hat  u  B_hat x A_hat`` with ``A_hat``, ``B_hat`` the unions over levels.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .graph import in_degrees, out_neighbours, transition_matrix


# --------------------------------------------------------------------------------------
# Rank-one factors of Delta Q
# --------------------------------------------------------------------------------------

def rank_one_insert(Q, d, i, j):
    """Theorem 1, eq (18): Delta Q = u v^T for inserting i -> j with i, j in V."""
    n = Q.shape[0]
    u = np.zeros(n)
    if d[j] == 0:
        u[j] = 1.0
        v = np.zeros(n)
        v[i] = 1.0
    else:
        u[j] = 1.0 / (d[j] + 1)
        v = -Q[j, :].copy()
        v[i] += 1.0
    return u, v


def rank_one_delete(Q, d, i, j):
    """Theorem 9: Delta Q = u v^T for deleting the existing edge i -> j."""
    n = Q.shape[0]
    u = np.zeros(n)
    if d[j] == 1:
        u[j] = 1.0
        v = np.zeros(n)
        v[i] = -1.0
    else:
        u[j] = 1.0 / (d[j] - 1)
        v = Q[j, :].copy()
        v[i] -= 1.0
    return u, v


def indicator(n, I):
    e = np.zeros(n)
    e[np.asarray(I, dtype=np.int64)] = 1.0
    return e


def rank_one_block(Q, d, I, j, op):
    """Table 2, rows (C0) insert / delete: one rank-one Delta Q for the delta edges
    ``{(i, j) : i in I}`` that share the sink j."""
    n = Q.shape[0]
    delta = len(I)
    eI = indicator(n, I)
    Qj = Q[j, :]
    if sp.issparse(Qj):
        Qj = np.asarray(Qj.todense()).ravel()
    u = np.zeros(n)
    if op > 0:
        if d[j] == 0:
            u[j] = 1.0
            v = eI / delta
        else:
            u[j] = delta / (d[j] + delta)
            v = eI / delta - Qj
    else:
        if d[j] == delta:
            u[j] = 1.0
            v = -eI / delta
        else:
            u[j] = delta / (d[j] - delta)
            v = Qj - eI / delta
    return u, v


# --------------------------------------------------------------------------------------
# gamma (or w) of the rank-one Sylvester equation
# --------------------------------------------------------------------------------------

def w_direct(Q, S, u, v):
    """Theorem 2, eq (20): ``w = y + (lambda / 2) u`` with ``z = S v``, ``y = Q z``,
    ``lambda = v^T z``. Valid for any S (does not use the fixed-point identity)."""
    z = S @ v
    y = Q @ z
    lam = float(v @ z)
    return y + 0.5 * lam * u


def gamma_closed_parts(QSI, Sj, SII, Sjj, dj, delta, j, C, op):
    """The arithmetic of the closed-form gamma, from its ingredients:
    ``QSI = Q S[:, I]`` (old Q), ``Sj = S[:, j]``, ``SII = S_{I,I}``, ``Sjj = S_jj``,
    ``dj`` the integer in-degree of j before the update and ``delta = |I|``.

    ``lambda = S_II / delta^2 + S_jj / C - (2 / delta) (Q S[:, I])_j - 1/C + 1`` (eq (29b),
    Table 2). Insertion: eq (29aa) when d_j = 0, eq (29bb) when d_j > 0. Deletion: the
    gamma of Theorem 9, with the Table 2 reading d_j = delta / d_j > delta.
    """
    n = QSI.shape[0]
    ej = np.zeros(n)
    ej[j] = 1.0
    lam = SII / delta ** 2 + Sjj / C - (2.0 / delta) * QSI[j] - 1.0 / C + 1.0
    if op > 0:
        if dj == 0:
            return QSI / delta + SII / (2.0 * delta ** 2) * ej
        f = delta / (dj + delta)
        return f * (QSI / delta - Sj / C
                    + (lam * delta / (2.0 * (dj + delta)) + 1.0 / C - 1.0) * ej)
    if dj == delta:
        return -QSI / delta + SII / (2.0 * delta ** 2) * ej
    f = delta / (dj - delta)
    return f * (Sj / C - QSI / delta
                + (lam * delta / (2.0 * (dj - delta)) - 1.0 / C + 1.0) * ej)


def gamma_closed(Q, S, d, I, j, C, op):
    """Closed-form gamma with ``M = sum_k C^(k+1) Qt^k e_j gamma^T (Qt^T)^k``.

    Unit updates (|I| = 1): Theorem 3, eqs (29aa), (29bb), (29b) for insertion and the
    gamma of Theorem 9 for deletion. Blocks: Table 2, rows (C0) insert / delete. These use
    eq (33), ``Q S Q[j,:]^T = (S[:, j] - (1 - C) e_j) / C``, so they assume S is the exact
    SimRank of the old graph.
    """
    I = np.asarray(I, dtype=np.int64)
    SI = S[:, I].sum(axis=1)                    # S[:, I]
    SII = float(S[np.ix_(I, I)].sum())          # S_{I,I}
    return gamma_closed_parts(Q @ SI, S[:, j], SII, float(S[j, j]), int(d[j]), len(I), j,
                              C, op)


def c2_z(Sj, Sjj, dj, delta, j, C):
    """Eq (60) and Table 2 row (C2):
    ``z = (1/(2C(d_j+delta)) (delta S_jj - (delta - C)(1 - C)) + (1 - C)/C) e_j - S[:, j]/C``."""
    n = Sj.shape[0]
    ej = np.zeros(n)
    ej[j] = 1.0
    return ((delta * Sjj - (delta - C) * (1.0 - C)) / (2.0 * C * (dj + delta))
            + (1.0 - C) / C) * ej - Sj / C


def gamma_from_direct(Q, S, u, v, j):
    """gamma of the direct form: ``C u w^T = C e_j (u_j w)^T``."""
    return u[j] * w_direct(Q, S, u, v)


# --------------------------------------------------------------------------------------
# Series vectors and Inc-uSR (Algorithm 1)
# --------------------------------------------------------------------------------------

def series(Q, u, v, xi0, eta0, C, K):
    """Eq (16a) as written in Algorithm 1: ``xi_{k+1} = C Q xi_k + C (v^T xi_k) u`` and
    ``eta_{k+1} = Q eta_k + (v^T eta_k) u`` (that is, multiplication by Qt = Q + u v^T),
    for k = 0..K-1. Returns the panels Xi, H with columns k = 0..K."""
    n = Q.shape[0]
    Xi = np.zeros((n, K + 1))
    H = np.zeros((n, K + 1))
    Xi[:, 0] = xi0
    H[:, 0] = eta0
    for k in range(K):
        Xi[:, k + 1] = C * (Q @ Xi[:, k]) + C * float(v @ Xi[:, k]) * u
        H[:, k + 1] = Q @ H[:, k] + float(v @ H[:, k]) * u
    return Xi, H


def inc_usr(Q, S, d, i, j, C, K, op=1, form="closed"):
    """Inc-uSR (Algorithm 1; deletion by Theorem 9) for an edge between existing nodes.

    Returns ``(S_new, info)`` with ``info`` holding u, v, gamma, Xi, H and M_K.
    ``form="closed"`` uses Theorem 3 / 9; ``form="direct"`` uses Theorem 2.
    """
    if op > 0:
        u, v = rank_one_insert(Q, d, i, j)
    else:
        u, v = rank_one_delete(Q, d, i, j)
    if form == "closed":
        gamma = gamma_closed(Q, S, d, [i], j, C, op)
    else:
        gamma = gamma_from_direct(Q, S, u, v, j)
    n = Q.shape[0]
    xi0 = np.zeros(n)
    xi0[j] = C
    Xi, H = series(Q, u, v, xi0, gamma, C, K)
    M = Xi @ H.T                                  # M_K = sum_k xi_k eta_k^T
    return S + M + M.T, dict(u=u, v=v, gamma=gamma, Xi=Xi, H=H, M=M)


def inc_block(Q, S, d, I, j, C, K, op, form="closed"):
    """Table 2, rows (C0): one block of delta edges sharing the sink j, both ends in V."""
    u, v = rank_one_block(Q, d, I, j, op)
    if form == "closed":
        gamma = gamma_closed(Q, S, d, I, j, C, op)
    else:
        gamma = gamma_from_direct(Q, S, u, v, j)
    n = Q.shape[0]
    xi0 = np.zeros(n)
    xi0[j] = C
    Xi, H = series(Q, u, v, xi0, gamma, C, K)
    M = Xi @ H.T
    return S + M + M.T, dict(u=u, v=v, gamma=gamma, Xi=Xi, H=H, M=M)


def truncation_bound(C, K, u, w):
    """Tail of M past K: ``|| sum_{k>K} C^(k+1) Qt^k u w^T Qt^Tk ||_max``
    ``<= sum_{k>K} C^(k+1) ||u||_inf ||w||_inf = C^(K+2)/(1-C) ||u||_inf ||w||_inf``
    (Qt^k does not increase the max-norm since its rows sum to at most 1), so
    ``||Delta S_K - Delta S||_max <= 2 C^(K+2)/(1-C) ||u||_inf ||w||_inf``."""
    return 2.0 * C ** (K + 2) / (1.0 - C) * float(np.max(np.abs(u))) * float(np.max(np.abs(w)))


# --------------------------------------------------------------------------------------
# Node insertions (section 6): C1, C2, C3, unit and block forms
# --------------------------------------------------------------------------------------

def grow(S, extra):
    n = S.shape[0]
    out = np.zeros((n + extra, n + extra))
    out[:n, :n] = S
    return out


def c1_block(Q, S, I, C):
    """Theorem 8 (Algorithm 3, Inc-uSR-C1) and Table 2 row (C1): new sink j = n with
    in-edges from the existing nodes I. ``y = (C / delta) Q S[:, I]`` borders S and the
    corner is ``(C / delta^2) S_{I,I} + 1 - C``."""
    I = np.asarray(I, dtype=np.int64)
    delta = len(I)
    n = S.shape[0]
    SI = S[:, I].sum(axis=1)
    y = (C / delta) * (Q @ SI)
    out = grow(S, 1)
    out[:n, n] = y
    out[n, :n] = y
    out[n, n] = (C / delta ** 2) * float(S[np.ix_(I, I)].sum()) + 1.0 - C
    return out


def c2_block(Q, S, d, delta, j, C, K):
    """Theorems 5-7 (Algorithm 4, Inc-uSR-C2) and Table 2 row (C2): delta new sources
    ``n..n+delta-1`` pointing to the existing sink j.

    ``Qh = Q - (delta / (d_j + delta)) e_j Q[j, :]``;
    ``z = (1/(2C(d_j+delta)) (delta S_jj - (delta - C)(1 - C)) + (1 - C)/C) e_j - S[:, j]/C``;
    ``M = sum_{k=0}^{K} C^k Qh^k e_j z^T (Qh^T)^k``; the old block becomes
    ``S + (C delta / (d_j + delta)) (M + M^T)`` and the new nodes get ``(1 - C) I_delta``.
    """
    n = S.shape[0]
    dj = int(d[j])
    Qh = Q.copy()
    Qh[j, :] -= (delta / (dj + delta)) * Q[j, :]
    ej = np.zeros(n)
    ej[j] = 1.0
    z = c2_z(S[:, j], float(S[j, j]), dj, delta, j, C)
    Xi = np.zeros((n, K + 1))
    H = np.zeros((n, K + 1))
    Xi[:, 0] = ej
    H[:, 0] = z
    for k in range(K):
        Xi[:, k + 1] = C * (Qh @ Xi[:, k])
        H[:, k + 1] = Qh @ H[:, k]
    M = Xi @ H.T
    out = grow(S, delta)
    out[:n, :n] = S + (C * delta / (dj + delta)) * (M + M.T)
    for t in range(delta):
        out[n + t, n + t] = 1.0 - C
    return out, dict(z=z, Xi=Xi, H=H, M=M, Qh=Qh)


def c3_block(S, delta, C):
    """Algorithm 5 (Inc-uSR-C3) and Table 2 row (C3): delta new sources ``n..n+delta-1``
    and a new sink ``n+delta`` form a separate component; its block is
    ``diag((1 - C) I_delta, (1 - C)(1 + C/delta))`` (``1 - C^2`` when delta = 1)."""
    n = S.shape[0]
    out = grow(S, delta + 1)
    for t in range(delta):
        out[n + t, n + t] = 1.0 - C
    out[n + delta, n + delta] = (1.0 - C) * (1.0 + C / delta)
    return out


# --------------------------------------------------------------------------------------
# Affected areas (Theorem 4)
# --------------------------------------------------------------------------------------

def _expand(out_nbrs, members):
    hit = set()
    for x in members:
        hit.update(int(b) for b in out_nbrs[x])
    return hit


def aff_sets(out_old, out_new, supp_I, supp_j, j, K):
    """Affected-area sets of Theorem 4 (eqs (39)-(41)) with the readings of this module.

    ``supp_I``: nodes y with ``S[i, y] != 0`` for some i in I (the union over I);
    ``supp_j``: nodes y with ``S[j, y] != 0`` when F2 applies, else ``None``.

    ``F1 = O_old(supp_I)``, ``F2 = supp_j`` (or empty), ``A_0 = {j}``,
    ``B_0 = F1 | F2 | {j}``; for k >= 1, ``A_k = O_new(A_0 | .. | A_{k-1})`` and
    ``B_k = O_new(B_0 | .. | B_{k-1})`` (out-neighbours in the new graph of the
    projections of the support of M_{k-1}). Returns sorted lists A, B per level and the
    unions ``A_hat``, ``B_hat``.
    """
    F1 = _expand(out_old, supp_I)
    F2 = set() if supp_j is None else set(int(y) for y in supp_j)
    A = [{int(j)}]
    B = [F1 | F2 | {int(j)}]
    UA = set(A[0])
    UB = set(B[0])
    for _k in range(1, K + 1):
        Ak = _expand(out_new, UA)
        Bk = _expand(out_new, UB)
        A.append(Ak)
        B.append(Bk)
        UA |= Ak
        UB |= Bk
    srt = lambda s: np.asarray(sorted(s), dtype=np.int64)
    return [srt(a) for a in A], [srt(b) for b in B], srt(UA), srt(UB)


def aff_pairs(A_hat, B_hat, n):
    """Boolean n x n mask of ``A_hat x B_hat  u  B_hat x A_hat``."""
    a = np.zeros(n, dtype=bool)
    b = np.zeros(n, dtype=bool)
    a[A_hat] = True
    b[B_hat] = True
    return np.outer(a, b) | np.outer(b, a)


def aff_pair_count(A_hat, B_hat):
    """|A x B  u  B x A| = 2 |A| |B| - |A & B|^2."""
    inter = np.intersect1d(A_hat, B_hat).size
    return 2 * len(A_hat) * len(B_hat) - inter * inter


def aff_for_update(n, src, dst, S, I, j, op, K, supp_eps=0.0):
    """AFF sets for the block ``{(i, j) : i in I}`` (op +1 insert, -1 delete) between
    existing nodes, with supports taken from the oracle's own S (``|S| > supp_eps``).

    F2 is empty when row j of Q is empty before an insertion (d_j = 0) or after a deletion
    (d_j = delta), following Theorem 4's last sentence and the Table 2 reading."""
    delta = len(I)
    d = in_degrees(n, src, dst)
    es = set(zip(np.asarray(src).tolist(), np.asarray(dst).tolist()))
    if op > 0:
        es2 = es | {(int(i), int(j)) for i in I}
        f2 = d[j] > 0
    else:
        es2 = es - {(int(i), int(j)) for i in I}
        f2 = d[j] > delta
    s2 = np.asarray([a for a, _ in es2], dtype=np.int64)
    d2 = np.asarray([b for _, b in es2], dtype=np.int64)
    out_old = out_neighbours(n, src, dst)
    out_new = out_neighbours(n, s2, d2)
    rows = np.abs(S[np.asarray(I, dtype=np.int64), :]) > supp_eps
    supp_I = np.nonzero(rows.any(axis=0))[0]
    supp_j = np.nonzero(np.abs(S[j, :]) > supp_eps)[0] if f2 else None
    return aff_sets(out_old, out_new, supp_I, supp_j, j, K)


# --------------------------------------------------------------------------------------
# Batch updates (section 8: net update, similar-sink partition, Table 2, Algorithm 6)
# --------------------------------------------------------------------------------------

def net_update(bi, bj, bop):
    """Net update by counting: +1 per insertion and -1 per deletion of each edge key; keys
    with nonzero count form Delta G_net. Returns ``(plus, minus)`` lists of ``(i, j)``
    sorted by (j, i). A net count outside {-1, 0, +1} is rejected."""
    cnt = {}
    for i, j, op in zip(np.asarray(bi).tolist(), np.asarray(bj).tolist(),
                        np.asarray(bop).tolist()):
        cnt[(i, j)] = cnt.get((i, j), 0) + (1 if op > 0 else -1)
    plus, minus = [], []
    for k, c in cnt.items():
        if c == 1:
            plus.append(k)
        elif c == -1:
            minus.append(k)
        elif c != 0:
            raise ValueError(f"net count {c} for edge {k}")
    key = lambda e: (e[1], e[0])
    return sorted(plus, key=key), sorted(minus, key=key)


def sink_blocks(edges):
    """Partition by "similar sink edges": one block per sink, sources ascending."""
    blocks = []
    for (i, j) in edges:
        if blocks and blocks[-1][1] == j:
            blocks[-1][0].append(i)
        else:
            blocks.append(([i], j))
    return blocks


def plan_batch(n, src, dst, bi, bj, bop, max_sources=None):
    """Algorithm 6 planning with the readings: deletion blocks first (sinks ascending),
    then insertion blocks (sinks ascending); each insertion block is split at the time it
    is processed into sources already in V (processed first) and sources not yet in V;
    a node joins V when a processed block creates it. Every block is applied whole, as one
    Table 2 update, whatever its number of sources.

    ``max_sources`` (off by default) instead takes a block of more sources as consecutive
    blocks of at most that many (sources ascending) with the same sink. Consecutive Table 2
    updates of one sink compose to the update of their union, so such a split reaches the
    same S as K grows; at a finite K each part has its own truncation. It exists only to
    check that composition.

    New node ids must be exactly ``n .. n + N - 1``. Returns a list of dicts with keys
    ``case`` (0..3), ``op``, ``I`` (sorted sources), ``j``, ``dj`` (in-degree of j when the
    block is processed) and the final node count.
    """
    plus, minus = net_update(bi, bj, bop)
    ids = set()
    for (i, j) in plus + minus:
        for x in (i, j):
            if x >= n:
                ids.add(x)
    n_new = n + len(ids)
    if ids and (min(ids) != n or max(ids) != n_new - 1):
        raise ValueError("new node ids are not dense")
    es = set(zip(np.asarray(src).tolist(), np.asarray(dst).tolist()))
    for (i, j) in minus:
        if (i, j) not in es:
            raise ValueError(f"delete of missing edge {(i, j)}")
    for (i, j) in plus:
        if (i, j) in es:
            raise ValueError(f"insert of existing edge {(i, j)}")
        if i == j:
            raise ValueError("self-loop")
    deg = {}
    for (_a, b) in es:
        deg[b] = deg.get(b, 0) + 1
    V = set(range(n))
    plan = []
    step = max_sources if max_sources else None
    for (I, j) in sink_blocks(minus):
        I = sorted(I)
        for lo in range(0, len(I), step or len(I)):
            part = I[lo:lo + step] if step else I
            plan.append(dict(case=0, op=-1, I=part, j=j, dj=deg.get(j, 0)))
            deg[j] = deg.get(j, 0) - len(part)
    for (I, j) in sink_blocks(plus):
        old = sorted(x for x in I if x in V)
        new = sorted(x for x in I if x not in V)
        for whole, in_v in ((old, True), (new, False)):
            for lo in range(0, len(whole), step or max(len(whole), 1)):
                part = whole[lo:lo + step] if step else whole
                j_in = j in V
                case = {(True, True): 0, (True, False): 1, (False, True): 2,
                        (False, False): 3}[(in_v, j_in)]
                plan.append(dict(case=case, op=1, I=part, j=j, dj=deg.get(j, 0)))
                deg[j] = deg.get(j, 0) + len(part)
                V.update(part)
                V.add(j)
    return plan, n_new


def inc_bsr(n, src, dst, S, bi, bj, bop, C, K, form="closed", max_sources=None):
    """Inc-bSR (Algorithm 6) evaluated densely block by block with Table 2.

    New-node blocks assume the new ids of a block are the next ids in processing order;
    to keep ids as given by the caller, S is first grown to the final node count with
    every not-yet-created node isolated (diagonal 1 - C, which is the SimRank of an
    isolated node) and the block formulas then act on the grown matrices.
    """
    plan, n_new = plan_batch(n, src, dst, bi, bj, bop, max_sources=max_sources)
    S = grow(S, n_new - n)
    for t in range(n, n_new):
        S[t, t] = 1.0 - C
    es = set(zip(np.asarray(src).tolist(), np.asarray(dst).tolist()))
    for blk in plan:
        s_arr = np.asarray([a for a, _ in es], dtype=np.int64)
        d_arr = np.asarray([b for _, b in es], dtype=np.int64)
        Q = transition_matrix(n_new, s_arr, d_arr, dense=True)
        d = in_degrees(n_new, s_arr, d_arr)
        I, j, case, op = blk["I"], blk["j"], blk["case"], blk["op"]
        if case == 0:
            S, _ = inc_block(Q, S, d, I, j, C, K, op, form)
        elif case == 1:
            S = _embed_c1(Q, S, I, j, C)
        elif case == 2:
            S = _embed_c2(Q, S, d, I, j, C, K)
        else:
            S = _embed_c3(S, I, j, C)
        for i in I:
            if op > 0:
                es.add((i, j))
            else:
                es.remove((i, j))
    return S, plan


def _embed_c1(Q, S, I, j, C):
    # Table 2 (C1) with the new sink j placed at its own id inside the grown matrix: the
    # block formula acts on the existing nodes, and row/column j (isolated so far) becomes
    # the border.
    keep = np.asarray([x for x in range(S.shape[0]) if x != j], dtype=np.int64)
    Ssub = S[np.ix_(keep, keep)]
    Qsub = Q[np.ix_(keep, keep)]
    pos = {x: p for p, x in enumerate(keep.tolist())}
    out = c1_block(Qsub, Ssub, [pos[i] for i in I], C)
    S = S.copy()
    S[keep, j] = out[:-1, -1]
    S[j, keep] = out[-1, :-1]
    S[j, j] = out[-1, -1]
    return S


def _embed_c2(Q, S, d, I, j, C, K):
    keep = np.asarray([x for x in range(S.shape[0]) if x not in set(I)], dtype=np.int64)
    pos = {x: p for p, x in enumerate(keep.tolist())}
    Qsub = Q[np.ix_(keep, keep)]
    Ssub = S[np.ix_(keep, keep)]
    dsub = d[keep]
    out, _ = c2_block(Qsub, Ssub, dsub, len(I), pos[j], C, K)
    S = S.copy()
    S[np.ix_(keep, keep)] = out[:len(keep), :len(keep)]
    for i in I:
        S[i, :] = 0.0
        S[:, i] = 0.0
        S[i, i] = 1.0 - C
    return S


def _embed_c3(S, I, j, C):
    S = S.copy()
    delta = len(I)
    for x in list(I) + [j]:
        S[x, :] = 0.0
        S[:, x] = 0.0
    for i in I:
        S[i, i] = 1.0 - C
    S[j, j] = (1.0 - C) * (1.0 + C / delta)
    return S


# --------------------------------------------------------------------------------------
# Memory-efficient column mode (section 7, Algorithm 7 Inc-SR-All-P)
# --------------------------------------------------------------------------------------

def delta_columns_c0(n, src, dst, i, j, cols, C, K, K_ps):
    """Columns ``Delta S[:, x]`` (x in ``cols``) for inserting i -> j between existing
    nodes, the way Algorithm 7 computes them in linear memory: PartialSim gives the old
    columns S[:, i] and S[:, j] (depth ``K_ps``), gamma follows Table 4's lines, the series
    vectors follow eq (16a), and eq (71) assembles
    ``Delta S[:, x] = M_K[:, x] + M_K[x, :]^T = sum_k (eta_k[x] xi_k + xi_k[x] eta_k)``.

    Returns an ``n x len(cols)`` array.
    """
    from .simrank import partial_sim
    Q = transition_matrix(n, src, dst)
    d = in_degrees(n, src, dst)
    Si = partial_sim(Q, i, K_ps, C)
    Sj = partial_sim(Q, j, K_ps, C)
    w = Q @ Si
    lam = Si[i] + Sj[j] / C - 2.0 * w[j] - 1.0 / C + 1.0
    ej = np.zeros(n)
    ej[j] = 1.0
    Qd = Q
    if d[j] == 0:
        u = ej.copy()
        vvec = np.zeros(n)
        vvec[i] = 1.0
        gamma = w + 0.5 * Si[i] * ej
    else:
        u = ej / (d[j] + 1)
        vvec = -np.asarray(Qd[j, :].todense()).ravel()
        vvec[i] += 1.0
        gamma = (w - Sj / C + (lam / (2.0 * (d[j] + 1)) + (1.0 - C) / C) * ej) / (d[j] + 1)
    xi = C * ej
    eta = gamma.copy()
    cols = np.asarray(cols, dtype=np.int64)
    m = np.outer(xi, eta[cols])          # columns of M_0: eta_0[x] xi_0
    nn = np.outer(eta, xi[cols])         # rows of M_0 transposed: xi_0[x] eta_0
    for _k in range(K):
        xi = C * (Q @ xi) + C * float(vvec @ xi) * u
        eta = Q @ eta + float(vvec @ eta) * u
        m += np.outer(xi, eta[cols])
        nn += np.outer(eta, xi[cols])
    return m + nn


def delta_columns_batch(n, src, dst, bi, bj, bop, cols, C, K, K_ps):
    """Columns ``Delta S[:, x]`` (x in ``cols``) of a batch of edge insertions and deletions
    between existing nodes, block by block in linear memory: the plan of Algorithm 6
    (net update, deletions first, sink-grouped blocks) with the column method of Algorithm 7
    inside each block. For block (I, j, op) on the graph as the earlier blocks left it,
    PartialSim (depth ``K_ps``) gives ``S[:, I] = sum_{i in I} S[:, i]`` and ``S[:, j]``;
    Table 2 row (C0) gives u, v and gamma; the series of eq (16a) gives xi_k, eta_k; and
    eq (71) adds ``sum_k (eta_k[x] xi_k + xi_k[x] eta_k)`` to column x. Then the block's
    edges are applied. A batch that creates nodes raises ValueError.

    Returns an ``n x len(cols)`` array.
    """
    from .simrank import partial_sim
    plan, n_new = plan_batch(n, src, dst, bi, bj, bop)
    if n_new != n or any(b["case"] != 0 for b in plan):
        raise ValueError("every edge of the batch must join existing nodes")
    cols = np.asarray(cols, dtype=np.int64)
    s_arr = np.asarray(src, dtype=np.int64)
    d_arr = np.asarray(dst, dtype=np.int64)
    out = np.zeros((n, len(cols)))
    for blk in plan:
        Q = transition_matrix(n, s_arr, d_arr)
        d = in_degrees(n, s_arr, d_arr)
        I, j, op = list(blk["I"]), blk["j"], blk["op"]
        SI = np.zeros(n)
        for i in I:
            SI += partial_sim(Q, i, K_ps, C)
        Sj = partial_sim(Q, j, K_ps, C)
        gamma = gamma_closed_parts(Q @ SI, Sj, float(SI[I].sum()), float(Sj[j]), int(d[j]),
                                   len(I), j, C, op)
        u, v = rank_one_block(Q, d, I, j, op)
        xi = np.zeros(n)
        xi[j] = C
        eta = gamma
        for k in range(K + 1):
            out += np.outer(xi, eta[cols]) + np.outer(eta, xi[cols])
            if k < K:
                xi, eta = (C * (Q @ xi) + C * float(v @ xi) * u,
                           Q @ eta + float(v @ eta) * u)
        # the block's edges i -> j, i in I
        if op > 0:
            s_arr = np.concatenate([s_arr, np.asarray(I, dtype=np.int64)])
            d_arr = np.concatenate([d_arr, np.full(len(I), j, dtype=np.int64)])
        else:
            drop = (d_arr == j) & np.isin(s_arr, np.asarray(I, dtype=np.int64))
            s_arr, d_arr = s_arr[~drop], d_arr[~drop]
    return out


def inc_sr_all_p_column(n, src, dst, S_col_x, x, edges, C, K, K_ps=None):
    """Algorithm 7 (Inc-SR-All-P) for one column x over a sequence of insertions ``edges``
    (each ``(i, j)``; new nodes take the next ids), with PartialSim at depth K as printed
    (``K_ps`` sets another PartialSim depth; the series keeps depth K).

    Returns the new column (length = final node count). With ``S_col_x`` zero it returns
    the column of Delta S (the new nodes' entries included)."""
    from .simrank import partial_sim
    Kp = K if K_ps is None else K_ps
    col = np.array(S_col_x, dtype=np.float64, copy=True)
    s = list(np.asarray(src).tolist())
    t = list(np.asarray(dst).tolist())
    cur_n = n
    for (i, j) in edges:
        Q = transition_matrix(cur_n, s, t)
        d = in_degrees(cur_n, s, t)
        i_in, j_in = i < cur_n, j < cur_n
        if i_in and j_in:                                   # case C0
            Si = partial_sim(Q, i, Kp, C)
            Sj = partial_sim(Q, j, Kp, C)
            w = Q @ Si
            lam = Si[i] + Sj[j] / C - 2.0 * w[j] - 1.0 / C + 1.0
            ej = np.zeros(cur_n)
            ej[j] = 1.0
            if d[j] == 0:
                u = ej.copy()
                vv = np.zeros(cur_n)
                vv[i] = 1.0
                gamma = w + 0.5 * Si[i] * ej
            else:
                u = ej / (d[j] + 1)
                vv = -np.asarray(Q[j, :].todense()).ravel()
                vv[i] += 1.0
                gamma = (w - Sj / C + (lam / (2.0 * (d[j] + 1)) + (1.0 - C) / C) * ej) / (
                    d[j] + 1)
            xi = C * ej
            eta = gamma.copy()
            m = C * gamma[x] * ej
            nn = C * ej[x] * gamma
            for _k in range(K):
                xi = C * (Q @ xi) + C * float(vv @ xi) * u
                eta = Q @ eta + float(vv @ eta) * u
                m = eta[x] * xi + m
                nn = xi[x] * eta + nn
            col = col + m + nn
        elif i_in and not j_in:                             # case C1
            Si = partial_sim(Q, i, Kp, C)
            y = C * (Q @ Si)
            if x == j:
                col = np.concatenate([y, [C * Si[i] + 1.0 - C]])
            else:
                col = np.concatenate([col, [y[x]]])
            cur_n += 1
        elif (not i_in) and j_in:                           # case C2
            if x == i:
                col = np.concatenate([np.zeros(cur_n), [1.0 - C]])
            else:
                Sj = partial_sim(Q, j, Kp, C)
                ej = np.zeros(cur_n)
                ej[j] = 1.0
                z = ((Sj[j] - (1.0 - C) ** 2) / (2.0 * C * (d[j] + 1)) + (1.0 - C) / C) * ej \
                    - Sj / C
                Qj = np.asarray(Q[j, :].todense()).ravel()
                xi = ej.copy()
                eta = z.copy()
                m = z[x] * ej
                nn = ej[x] * z
                for _k in range(K):
                    xi = C * (Q @ xi) - C / (d[j] + 1) * float(Qj @ xi) * ej
                    eta = Q @ eta - 1.0 / (d[j] + 1) * float(Qj @ eta) * ej
                    m = eta[x] * xi + m
                    nn = xi[x] * eta + nn
                col = np.concatenate([col + C / (d[j] + 1) * (m + nn), [0.0]])
            cur_n += 1
        else:                                               # case C3
            if x == i:
                col = np.concatenate([np.zeros(cur_n), [1.0 - C, 0.0]])
            elif x == j:
                col = np.concatenate([np.zeros(cur_n), [0.0, 1.0 - C * C]])
            else:
                col = np.concatenate([col, [0.0, 0.0]])
            cur_n += 2
        s.append(i)
        t.append(j)
    return col
