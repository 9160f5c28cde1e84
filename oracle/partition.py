"""All-pairs SimRank over a partitioned graph (Example 1.1, decentralised retrieval): the graph
is cut into blocks, S of the blocks' own edges is block diagonal and each block is computed on
its own, and the edges across blocks are applied to it as one batch of insertions.

* ``bfs_partition``   the partitioner both sides use (METIS is not available): blocks of at
                      most ceil(n / parts) nodes grown breadth first over the undirected graph.
                      A block starts at the smallest unassigned id; neighbours are scanned in
                      ascending id; a block that is full stops at once, and one whose search
                      runs dry continues from the smallest unassigned id.
* ``block_simrank``   S of the blocks' own edges: the fixed point of eq (03a) of every block
                      computed on the block alone and placed on the diagonal.
* ``partitioned``     ``block_simrank``, then the cross-block edges (caller's order) by Inc-bSR
                      (Algorithm 6, Table 2).

Test infrastructure: only the test suite, the smoke check and the benchmark's CPU-baseline
leg import this module.
"""
from __future__ import annotations

from collections import deque

import numpy as np

from .graph import transition_matrix
from .incremental import inc_bsr
from .simrank import fixed_point


def bfs_partition(n, src, dst, parts):
    """Block label of every node by the rule in the module header."""
    cap = -(-n // parts)
    nbrs = [set() for _ in range(n)]
    for a, b in zip(np.asarray(src).tolist(), np.asarray(dst).tolist()):
        nbrs[a].add(b)
        nbrs[b].add(a)
    nbrs = [sorted(s) for s in nbrs]
    label = np.full(n, -1, dtype=np.int64)
    p, size, nxt = 0, 0, 0
    while True:
        while nxt < n and label[nxt] >= 0:
            nxt += 1
        if nxt == n:
            break
        label[nxt] = p
        size += 1
        queue = deque([nxt])
        full = size == cap
        while queue and not full:
            u = queue.popleft()
            for v in nbrs[u]:
                if label[v] < 0:
                    label[v] = p
                    size += 1
                    queue.append(v)
                    if size == cap:
                        full = True
                        break
        if full:
            p, size = p + 1, 0
    return label


def block_simrank(n, src, dst, label, C):
    """Dense S of the edges inside blocks: each block's fixed point on its own nodes."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    label = np.asarray(label)
    S = np.zeros((n, n))
    for p in np.unique(label):
        nodes = np.nonzero(label == p)[0]
        loc = np.full(n, -1, dtype=np.int64)
        loc[nodes] = np.arange(len(nodes))
        inside = (label[src] == p) & (label[dst] == p)
        Sb = fixed_point(transition_matrix(len(nodes), loc[src[inside]], loc[dst[inside]]), C)
        S[np.ix_(nodes, nodes)] = Sb
    return S


def partitioned(n, src, dst, label, C, K):
    """Example 1.1: S of the blocks, then the cross-block edges as one Inc-bSR batch."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    label = np.asarray(label)
    inside = label[src] == label[dst]
    S = block_simrank(n, src[inside], dst[inside], label, C)
    cs, cd = src[~inside], dst[~inside]
    S, _ = inc_bsr(n, src[inside], dst[inside], S, cs, cd, np.ones(len(cs), dtype=np.int64),
                   C, K)
    return S
