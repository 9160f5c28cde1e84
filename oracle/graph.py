"""Backward transition matrix Q of a digraph (section 3.1, definition under eq (03a)).

``Q[a, x] = 1 / indeg(a)`` when the edge ``x -> a`` exists, else 0; a node without
in-edges has an all-zero row. For a weighted graph (used only by the adjoint, which the
paper does not cover) the row is normalised by the weights instead:
``Q[a, x] = w(x -> a) / sum of the weights of a's in-edges``.

In-degrees are integers counted from the edge list, never read back from the nonzeros of a
floating-point Q.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def in_degrees(n, src, dst):
    """Integer in-degree of every node."""
    return np.bincount(np.asarray(dst, dtype=np.int64), minlength=n).astype(np.int64)


def out_neighbours(n, src, dst):
    """List of out-neighbour arrays per node (node -> nodes it points to)."""
    order = np.argsort(np.asarray(src, dtype=np.int64), kind="stable")
    s = np.asarray(src, dtype=np.int64)[order]
    d = np.asarray(dst, dtype=np.int64)[order]
    ptr = np.searchsorted(s, np.arange(n + 1))
    return [d[ptr[v]:ptr[v + 1]] for v in range(n)]


def transition_matrix(n, src, dst, weight=None, dense=False):
    """Q as a scipy CSR matrix (or a dense array when ``dense``)."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    if weight is None:
        deg = in_degrees(n, src, dst)
        vals = 1.0 / deg[dst].astype(np.float64) if dst.size else np.zeros(0)
    else:
        w = np.asarray(weight, dtype=np.float64)
        wsum = np.bincount(dst, weights=w, minlength=n)
        vals = w / wsum[dst]
    Q = sp.csr_matrix((vals, (dst, src)), shape=(n, n))
    Q.sum_duplicates()
    return Q.toarray() if dense else Q


def edge_set(src, dst):
    return set(zip(np.asarray(src).tolist(), np.asarray(dst).tolist()))


def apply_edges(n, src, dst, upd_i, upd_j, upd_op, n_new=None):
    """Edge list after applying insertions (+1) and deletions (-1) in order.

    Returns ``(n', src', dst')`` with edges sorted by (dst, src). Raises on an invalid
    update (inserting an existing edge, deleting a missing one, a self-loop).
    """
    es = edge_set(src, dst)
    n2 = n if n_new is None else n_new
    for i, j, op in zip(np.asarray(upd_i).tolist(), np.asarray(upd_j).tolist(),
                        np.asarray(upd_op).tolist()):
        if i == j:
            raise ValueError("self-loop")
        if op > 0:
            if (i, j) in es:
                raise ValueError(f"edge {(i, j)} exists")
            es.add((i, j))
            n2 = max(n2, i + 1, j + 1)
        else:
            if (i, j) not in es:
                raise ValueError(f"edge {(i, j)} missing")
            es.remove((i, j))
    e = sorted(es, key=lambda t: (t[1], t[0]))
    s = np.asarray([a for a, _ in e], dtype=np.int32)
    d = np.asarray([b for _, b in e], dtype=np.int32)
    return n2, s, d
