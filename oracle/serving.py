"""Top-k single-source similarity search on SimRank scores (serving after updates; the
paper's effectiveness study ranks nodes by their similarity to a query the same way).

* ``topk``            the k nodes with the largest score in a query's column, best first,
                      ties to the smaller node id, the query itself optionally left out.
* ``precision_at_k``  the fraction of a returned list that lies in the true top-k.

Test infrastructure: only the test suite, the smoke check and the benchmark's CPU-baseline
leg import this module.
"""
from __future__ import annotations

import numpy as np


def topk(col, x, k, exclude_self=True):
    """Indices and values of the k largest entries of ``col`` (length n), best first, equal
    values ordered by ascending index, index ``x`` skipped when ``exclude_self``."""
    col = np.asarray(col, dtype=np.float64)
    ids = np.arange(len(col))
    keep = ids != x if exclude_self else np.ones(len(col), dtype=bool)
    ids = ids[keep]
    vals = col[keep]
    order = np.lexsort((ids, -vals))[:k]
    return ids[order], vals[order]


def precision_at_k(found, truth):
    """|found & truth| / |truth| for two lists of node ids."""
    truth = set(np.asarray(truth).tolist())
    return len(truth & set(np.asarray(found).tolist())) / max(len(truth), 1)
