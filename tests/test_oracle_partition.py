"""Pins of the partitioned all-pairs SimRank (Example 1.1) in the oracle: the partition rule
on a graph worked by hand and its size and cover properties, the block-diagonal S against the
fixed point of eq (03a) on the union of the blocks, and the pipeline against the fixed point
on the whole graph."""
import numpy as np
import pytest

import workloads as W
from oracle import graph as Gr
from oracle import incremental as OI
from oracle import partition as Pt
from oracle import simrank as O

C = 0.6


def test_partition_worked_by_hand():
    # undirected neighbours: 0-{3,5}, 1-{2}, 2-{1,4}, 3-{0,4}, 4-{2,3}, 5-{0}; cap = 3
    # block 0 from 0: 3, 5 (full); block 1 from 1: 2, then 4 (full)
    s = np.array([0, 5, 1, 2, 4, 3])
    d = np.array([3, 0, 2, 4, 3, 4])
    assert Pt.bfs_partition(6, s, d, 2).tolist() == [0, 1, 1, 0, 1, 0]
    # a block whose search runs dry continues from the smallest unassigned id
    s = np.array([0, 2])
    d = np.array([1, 3])
    assert Pt.bfs_partition(5, s, d, 2).tolist() == [0, 0, 0, 1, 1]


@pytest.mark.parametrize("seed", range(3))
def test_partition_sizes_and_cover(seed):
    n, parts = 203, 8
    s, d, _ = W.communities(n, 900, parts, 0.05, seed=600 + seed)
    lab = Pt.bfs_partition(n, s, d, parts)
    cap = -(-n // parts)
    counts = np.bincount(lab)
    assert lab.min() == 0 and len(counts) == -(-n // cap)
    assert np.all(counts[:-1] == cap) and 0 < counts[-1] <= cap
    assert np.array_equal(lab, Pt.bfs_partition(n, s, d, parts))


def test_block_simrank_is_the_fixed_point_of_the_blocks():
    n = 120
    s, d, _ = W.communities(n, 500, 4, 0.05, seed=610)
    lab = Pt.bfs_partition(n, s, d, 4)
    inside = lab[s] == lab[d]
    Sb = Pt.block_simrank(n, s[inside], d[inside], lab, C)
    Sf = O.fixed_point(Gr.transition_matrix(n, s[inside], d[inside]), C)
    assert np.abs(Sb - Sf).max() < 1e-14
    assert np.abs(Sb[lab[:, None] != lab[None, :]]).max() == 0.0


def test_partitioned_pipeline_reaches_the_fixed_point():
    n = 100
    s, d, _ = W.communities(n, 420, 4, 0.05, seed=620)
    lab = Pt.bfs_partition(n, s, d, 4)
    exact = O.fixed_point(Gr.transition_matrix(n, s, d), C)
    assert np.abs(Pt.partitioned(n, s, d, lab, C, 70) - exact).max() < 1e-11
    inside = lab[s] == lab[d]
    S0 = O.fixed_point(Gr.transition_matrix(n, s[inside], d[inside]), C)
    ref, plan = OI.inc_bsr(n, s[inside], d[inside], S0, s[~inside], d[~inside],
                           np.ones((~inside).sum(), dtype=np.int64), C, 15)
    S15 = Pt.partitioned(n, s, d, lab, C, 15)
    assert np.abs(S15 - ref).max() < 1e-13
    assert np.abs(S15 - exact).max() < len(plan) * 2 * C ** 17 / (1 - C)
