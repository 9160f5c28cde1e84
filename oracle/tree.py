"""All-pairs SimRank seeded from a spanning forest (Example 1.2, the batch-computation use of
the incremental method).

Steps, in the example's order:

1. ``bfs_forest``: a breadth-first spanning forest (a branching) of the digraph. Every node
   gets at most one tree in-edge, from the node that first reached it.
2. ``tree_simrank``: S of the forest alone by the example's closed form. On a forest every
   non-root has one in-neighbour (its parent), so ``Q^k (Q^T)^k [a][b]`` is 1 exactly when a
   and b have the same ancestor k levels up. Two nodes at different depths never do; two
   nodes at depth H whose lowest common ancestor is lambda edges up do for k = lambda .. H,
   which sums (eq (17)) to ``C^lambda (1 - C^(H - lambda + 1))``; nodes of different trees
   never meet, and score 0.
3. ``tree_seeded``: the remaining edges, in the caller's order, applied to S of the forest as
   one batch by Inc-bSR (Algorithm 6, Table 2).

The forest rule (fixed so that two implementations build the same forest): the nodes without
in-edges, which must be roots, are taken first in ascending id, then every node not reached
yet, in ascending id; each tree is grown breadth first, a node's out-neighbours being scanned
in ascending id.

Test infrastructure: only the test suite, the smoke check and the benchmark's CPU-baseline
leg import this module.
"""
from __future__ import annotations

from collections import deque

import numpy as np

from .graph import out_neighbours
from .incremental import inc_bsr


def bfs_forest(n, src, dst):
    """Parent (-1 for a root) and depth of every node in the breadth-first spanning forest
    described in the module header."""
    outs = out_neighbours(n, np.asarray(src, dtype=np.int64), np.asarray(dst, dtype=np.int64))
    parent = np.full(n, -1, dtype=np.int64)
    depth = np.zeros(n, dtype=np.int64)
    seen = np.zeros(n, dtype=bool)
    indeg = np.bincount(np.asarray(dst, dtype=np.int64), minlength=n)
    order = list(np.nonzero(indeg == 0)[0]) + list(np.nonzero(indeg > 0)[0])
    for r in order:
        if seen[r]:
            continue
        seen[r] = True
        queue = deque([r])
        while queue:
            u = queue.popleft()
            for v in sorted(outs[u]):
                if not seen[v]:
                    seen[v] = True
                    parent[v] = u
                    depth[v] = depth[u] + 1
                    queue.append(v)
    return parent, depth


def tree_simrank(parent, depth, C):
    """Dense S of the forest by Example 1.2's closed form: for a and b at the same depth H in
    one tree, lambda = edges from their lowest common ancestor down to a, and
    ``S[a][b] = C^lambda (1 - C^(H - lambda + 1))``; every other pair scores 0."""
    parent = np.asarray(parent, dtype=np.int64)
    depth = np.asarray(depth, dtype=np.int64)
    n = len(parent)
    S = np.zeros((n, n))
    for H in np.unique(depth):
        level = np.nonzero(depth == H)[0]
        for a in level:
            for b in level:
                x, y, lam = a, b, 0
                while x != y and x >= 0:
                    x, y, lam = parent[x], parent[y], lam + 1
                if x == y:
                    S[a, b] = C ** lam * (1.0 - C ** (H - lam + 1))
    return S


def tree_edges(n, src, dst, parent):
    """Boolean mask over the edge list: True for the forest's edges ``parent[v] -> v``."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    return parent[dst] == src


def tree_seeded(n, src, dst, C, K):
    """Example 1.2: S of the forest, then the other edges (caller's order) as one Inc-bSR
    batch of insertions. Returns the dense S after the batch."""
    parent, depth = bfs_forest(n, src, dst)
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    on = tree_edges(n, src, dst, parent)
    S = tree_simrank(parent, depth, C)
    rest_s, rest_d = src[~on], dst[~on]
    S, _ = inc_bsr(n, src[on], dst[on], S, rest_s, rest_d,
                   np.ones(len(rest_s), dtype=np.int64), C, K)
    return S
