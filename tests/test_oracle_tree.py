"""Pins of the forest-seeded all-pairs SimRank (Example 1.2) in the oracle: the forest rule on
a graph worked by hand and its breadth-first and branching properties on random graphs, the
closed form against the fixed point of eq (03a) on the forest, and the whole seeded pipeline
against the fixed point on the full graph."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

from oracle import graph as Gr
from oracle import simrank as O
from oracle import tree as T
import workloads as W

C = 0.6


def test_forest_worked_by_hand():
    # edges: 0->2, 0->1, 1->3, 2->3, 3->0, 4->3, 5->4, 2->5
    # root 0 (lowest id): depth 1 = {1, 2} (scanned in ascending id), 3 reached first from 1,
    # 5 from 2, then 4 from 5; 3 -> 0 and 2 -> 3 and 4 -> 3 are non-tree edges
    s = np.array([0, 0, 1, 2, 3, 4, 5, 2])
    d = np.array([2, 1, 3, 3, 0, 3, 4, 5])
    parent, depth = T.bfs_forest(6, s, d)
    assert parent.tolist() == [-1, 0, 0, 1, 5, 2]
    assert depth.tolist() == [0, 1, 1, 2, 3, 2]
    on = T.tree_edges(6, s, d, parent)
    assert on.tolist() == [True, True, True, False, False, False, True, True]
    # nodes without in-edges are roots first: 0 and 3, so 3 -> 2 is a tree edge
    parent, depth = T.bfs_forest(4, np.array([0, 3]), np.array([1, 2]))
    assert parent.tolist() == [-1, 0, 3, -1] and depth.tolist() == [0, 1, 1, 0]


@pytest.mark.parametrize("seed", range(4))
def test_forest_is_a_breadth_first_branching(seed):
    n = 120
    s, d = W.chung_lu(n, 500, seed=700 + seed)
    parent, depth = T.bfs_forest(n, s, d)
    es = set(zip(s.tolist(), d.tolist()))
    indeg = Gr.in_degrees(n, s, d)
    roots = np.nonzero(parent < 0)[0]
    assert all(depth[r] == 0 for r in roots)
    assert all(indeg[v] > 0 for v in range(n) if parent[v] >= 0)
    for v in range(n):
        if parent[v] >= 0:
            assert (int(parent[v]), v) in es
            assert depth[v] == depth[parent[v]] + 1
    # a node without in-edges is a root
    assert all(parent[v] < 0 for v in range(n) if indeg[v] == 0)
    assert T.tree_edges(n, s, d, parent).sum() == n - len(roots)
    # the first tree (lowest id without in-edges) holds exactly the nodes reachable from its
    # root, at their shortest distances
    r0 = int(np.nonzero(indeg == 0)[0][0])
    A = sp.csr_matrix((np.ones(len(s)), (s, d)), shape=(n, n))
    dist = shortest_path(A, indices=r0, unweighted=True)
    reach = np.isfinite(dist)
    root_of = np.arange(n)
    for v in np.argsort(depth, kind="stable"):
        if parent[v] >= 0:
            root_of[v] = root_of[parent[v]]
    assert np.array_equal(reach, root_of == r0)
    assert np.array_equal(depth[reach], dist[reach].astype(int))


@pytest.mark.parametrize("seed", range(4))
def test_closed_form_is_the_fixed_point_of_the_forest(seed):
    n = 90
    s, d = W.chung_lu(n, 240, seed=710 + seed)
    parent, depth = T.bfs_forest(n, s, d)
    on = T.tree_edges(n, s, d, parent)
    assert (parent < 0).sum() >= 2     # several trees: cross-tree pairs must score 0
    for c in (0.6, 0.8):
        Sf = O.fixed_point(Gr.transition_matrix(n, s[on], d[on]), c)
        assert np.abs(T.tree_simrank(parent, depth, c) - Sf).max() < 1e-14


def test_seeded_pipeline_reaches_the_fixed_point_of_the_graph():
    n = 60
    s, d = W.chung_lu(n, 260, seed=720)
    exact = O.fixed_point(Gr.transition_matrix(n, s, d), C)
    # deep series: each block drops less than C^(K+1) / (1 - C) of its Delta S
    S = T.tree_seeded(n, s, d, C, 70)
    assert np.abs(S - exact).max() < 1e-11
    # at K = 15 the error stays within the blocks' summed truncation bounds
    parent, _ = T.bfs_forest(n, s, d)
    blocks = len({int(x) for x in d[~T.tree_edges(n, s, d, parent)]})
    S15 = T.tree_seeded(n, s, d, C, 15)
    assert 0.0 < np.abs(S15 - exact).max() < blocks * 2 * C ** 17 / (1 - C)


def test_seeded_pipeline_equals_batch_from_the_forest_fixed_point():
    n = 50
    s, d = W.chung_lu(n, 200, seed=730)
    parent, depth = T.bfs_forest(n, s, d)
    on = T.tree_edges(n, s, d, parent)
    S0 = O.fixed_point(Gr.transition_matrix(n, s[on], d[on]), C)
    from oracle import incremental as OI
    ref, _ = OI.inc_bsr(n, s[on], d[on], S0, s[~on], d[~on],
                        np.ones((~on).sum(), dtype=np.int64), C, 15)
    assert np.abs(T.tree_seeded(n, s, d, C, 15) - ref).max() < 1e-13
