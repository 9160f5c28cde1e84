"""Pins of the oracle's batch path (section 8, Table 2, Algorithm 6): the paper's net-update
and similar-sink examples, Inc-bSR equal to recompute on random mixed batches, and the
memory-efficient column mode (Algorithm 7) equal to recompute."""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import graph as Gr
from oracle import incremental as I
from oracle import simrank as O

C = 0.6
HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "worked_examples.json")))


def test_paper_net_update_and_partition():
    g = GOLD["batch_example"]
    names = list(g["nodes_existing"]) + ["q", "p", "r"]      # new ids by first appearance
    idx = {x: p for p, x in enumerate(names)}
    bi = [idx[a] for a, _, _ in g["updates"]]
    bj = [idx[b] for _, b, _ in g["updates"]]
    bo = [op for _, _, op in g["updates"]]
    plus, minus = I.net_update(bi, bj, bo)
    nm = lambda e: [names[e[0]], names[e[1]]]
    assert sorted(map(nm, plus)) == sorted(g["net_plus"])
    assert sorted(map(nm, minus)) == sorted(g["net_minus"])
    # a graph on a..o that holds the deleted edge (f, b)
    n = 15
    src = [idx["f"], idx["a"], idx["c"]]
    dst = [idx["b"], idx["i"], idx["f"]]
    plan, n_new = I.plan_batch(n, src, dst, bi, bj, bo)
    assert n_new == 18
    got_plus = sorted(([names[x] for x in b["I"]], names[b["j"]]) for b in plan if b["op"] > 0)
    exp_plus = sorted((sorted(I_), j) for I_, j in g["plus_blocks"])
    assert got_plus == exp_plus
    got_minus = [([names[x] for x in b["I"]], names[b["j"]]) for b in plan if b["op"] < 0]
    assert got_minus == [(I_, j) for I_, j in g["minus_blocks"]]
    cases = {(tuple(names[x] for x in b["I"]), names[b["j"]]): b["case"] for b in plan}
    assert cases[(("q",), "i")] == 2           # new source into existing sink
    assert cases[(("j", "k"), "i")] == 0       # existing sources
    assert cases[(("p", "r"), "f")] == 2
    # deletions are planned before insertions
    assert plan[0]["op"] == -1


def test_net_update_rejects_double_insert():
    import pytest
    with pytest.raises(ValueError):
        I.net_update([0, 0], [1, 1], [1, 1])


def test_inc_bsr_matches_recompute():
    rng = np.random.default_rng(51)
    worst = 0.0
    for trial in range(25):
        n = int(rng.integers(6, 10))
        s, d = W.chung_lu(n, int(rng.integers(n, 2 * n)), seed=500 + trial)
        Q = Gr.transition_matrix(n, s, d)
        S = O.fixed_point(Q, C)
        b, cnt = W.batch_stream(n, s, d, 1, 6, 600 + trial, min_batch=3)
        bi, bj, bo = b[0]
        for form in ("closed", "direct"):
            Sn, plan = I.inc_bsr(n, s, d, S, bi, bj, bo, C, 80, form)
            plus, minus = I.net_update(bi, bj, bo)
            n2, s2, d2 = Gr.apply_edges(
                n, s, d, [e[0] for e in plus + minus], [e[1] for e in plus + minus],
                [1] * len(plus) + [-1] * len(minus), n_new=cnt[0])
            S2 = O.fixed_point(Gr.transition_matrix(n2, s2, d2), C)
            worst = max(worst, np.abs(Sn - S2).max())
    assert worst < 1e-13


def test_plan_blocks_cover_net_update_once():
    n = 300
    s, d = W.chung_lu(n, 1500, seed=61)
    batches, counts = W.batch_stream(n, s, d, 3, 300, 62)
    cur_s, cur_d, cur_n = s, d, n
    for (bi, bj, bo), nn in zip(batches, counts):
        plan, n_new = I.plan_batch(cur_n, cur_s, cur_d, bi, bj, bo)
        assert n_new == nn
        plus, minus = I.net_update(bi, bj, bo)
        got = sorted((i, b["j"], b["op"]) for b in plan for i in b["I"])
        exp = sorted([(i, j, 1) for i, j in plus] + [(i, j, -1) for i, j in minus])
        assert got == exp
        for b in plan:
            assert b["I"] == sorted(b["I"])
        cur_n, cur_s, cur_d = Gr.apply_edges(
            cur_n, cur_s, cur_d, [e[0] for e in plus + minus], [e[1] for e in plus + minus],
            [1] * len(plus) + [-1] * len(minus), n_new=nn)


def test_column_mode_matches_recompute():
    n = 60
    s, d = W.chung_lu(n, 240, seed=71)
    Q = Gr.transition_matrix(n, s, d)
    S = O.fixed_point(Q, C)
    i_s, j_s = W.insertion_stream(n, s, d, 3, seed=72)
    cur_s, cur_d = s.astype(np.int64), d.astype(np.int64)
    for i, j in zip(i_s.tolist(), j_s.tolist()):
        cols = [0, 3, i, j, 59]
        got = I.delta_columns_c0(n, cur_s, cur_d, i, j, cols, C, 70, 70)
        n2, s2, d2 = Gr.apply_edges(n, cur_s, cur_d, [i], [j], [1])
        S_new = O.fixed_point(Gr.transition_matrix(n2, s2, d2), C)
        S_old = O.fixed_point(Gr.transition_matrix(n, cur_s, cur_d), C)
        assert np.abs(got - (S_new - S_old)[:, cols]).max() < 1e-13
        cur_s, cur_d = s2.astype(np.int64), d2.astype(np.int64)


def test_algorithm7_column_all_cases():
    """Algorithm 7 with node insertions (C0-C3) for one carried column x, deep K."""
    n = 40
    s, d = W.chung_lu(n, 150, seed=81)
    Q = Gr.transition_matrix(n, s, d)
    S = O.fixed_point(Q, C)
    es = set(zip(s.tolist(), d.tolist()))
    edges = [(1, 2) if (1, 2) not in es else (2, 1), (5, n), (n + 1, 7), (n + 2, n + 3)]
    for x in (0, 7, n):
        if x >= n:
            continue
        col = I.inc_sr_all_p_column(n, s, d, S[:, x], x, edges, C, 70)
        n2, s2, d2 = Gr.apply_edges(n, s, d, [e[0] for e in edges], [e[1] for e in edges],
                                    [1] * len(edges))
        S2 = O.fixed_point(Gr.transition_matrix(n2, s2, d2), C)
        assert np.abs(col - S2[:, x]).max() < 1e-13


def _mixed_existing_batch(n, s, d, seed, n_ins=10, n_del=6, shared=3):
    """Insertions of non-edges (some sharing a sink) and deletions of existing edges,
    all between existing nodes."""
    g = W.rng(seed)
    es = set(zip(s.tolist(), d.tolist()))
    bi, bj, bo = [], [], []
    sink = int(g.integers(n))
    while len(bi) < n_ins:
        a = int(g.integers(n))
        b = sink if len(bi) < shared else int(g.integers(n))
        if a != b and (a, b) not in es and (a, b) not in zip(bi, bj):
            bi.append(a)
            bj.append(b)
            bo.append(1)
    for e in g.choice(len(s), size=n_del, replace=False).tolist():
        bi.append(int(s[e]))
        bj.append(int(d[e]))
        bo.append(-1)
    return bi, bj, bo


def test_column_batch_matches_recompute():
    """Algorithm 6's blocks with the column method inside (deep K and PartialSim depth):
    the summed Delta S columns equal the difference of the converged S of the two graphs."""
    n = 60
    s, d = W.chung_lu(n, 240, seed=73)
    bi, bj, bo = _mixed_existing_batch(n, s, d, seed=74)
    cols = [0, 3, bj[0], bi[0], 59]
    got = I.delta_columns_batch(n, s.astype(np.int64), d.astype(np.int64), bi, bj, bo, cols,
                                C, 70, 70)
    n2, s2, d2 = Gr.apply_edges(n, s, d, bi, bj, bo)
    S_new = O.fixed_point(Gr.transition_matrix(n2, s2, d2), C)
    S_old = O.fixed_point(Gr.transition_matrix(n, s, d), C)
    assert np.abs(got - (S_new - S_old)[:, cols]).max() < 1e-13


def test_column_batch_single_edge_is_the_unit_column_method():
    n = 60
    s, d = W.chung_lu(n, 240, seed=75)
    ii, jj = W.insertion_stream(n, s, d, 1, seed=76)
    i, j = int(ii[0]), int(jj[0])
    cols = [1, 2, i, j]
    a = I.delta_columns_batch(n, s.astype(np.int64), d.astype(np.int64), [i], [j], [1], cols,
                              C, 10, 30)
    b = I.delta_columns_c0(n, s.astype(np.int64), d.astype(np.int64), i, j, cols, C, 10, 30)
    assert np.abs(a - b).max() < 1e-15


def test_column_batch_equals_dense_inc_bsr_at_depth():
    """At deep K the column form of the batch and the dense Inc-bSR give the same Delta S
    columns (the dense form starts from the converged S)."""
    n = 60
    s, d = W.chung_lu(n, 240, seed=77)
    bi, bj, bo = _mixed_existing_batch(n, s, d, seed=78)
    cols = list(range(0, n, 7))
    S_old = O.fixed_point(Gr.transition_matrix(n, s, d), C)
    S_new, _ = I.inc_bsr(n, s.astype(np.int64), d.astype(np.int64), S_old, bi, bj, bo, C, 70)
    got = I.delta_columns_batch(n, s.astype(np.int64), d.astype(np.int64), bi, bj, bo, cols,
                                C, 70, 70)
    assert np.abs(got - (S_new - S_old)[:, cols]).max() < 1e-12


def test_column_batch_rejects_new_nodes():
    n = 20
    s, d = W.chung_lu(n, 60, seed=79)
    with pytest.raises(ValueError):
        I.delta_columns_batch(n, s, d, [1], [n], [1], [0], C, 5, 5)


def test_long_blocks_are_one_block_each():
    """Algorithm 6 applies a sink's whole block as one Table 2 update: 130 existing sources
    into sink 0 and 70 existing sources into the new sink 200 give two blocks."""
    n = 200
    src, dst = [1], [2]
    bi = list(range(3, 133))                      # 130 existing sources into sink 0
    bj = [0] * 130
    bi += list(range(10, 80))                     # 70 existing sources into the new sink 200
    bj += [200] * 70
    plan, n_new = I.plan_batch(n, src, dst, bi, bj, [1] * len(bi))
    assert n_new == 201
    assert [(b["case"], b["j"], len(b["I"]), b["dj"]) for b in plan] == \
        [(0, 0, 130, 0), (1, 200, 70, 0)]
    assert plan[0]["I"] == list(range(3, 133)) and plan[1]["I"] == list(range(10, 80))


def test_optional_split_takes_consecutive_blocks_of_one_sink():
    """With max_sources the same batch becomes consecutive blocks of at most 60 (sources
    ascending); a new sink's later parts find it existing (case C1 then C0)."""
    n = 200
    src, dst = [1], [2]
    bi = list(range(3, 133)) + list(range(10, 80))
    bj = [0] * 130 + [200] * 70
    plan, _ = I.plan_batch(n, src, dst, bi, bj, [1] * len(bi), max_sources=60)
    sizes = [(b["case"], b["j"], len(b["I"]), b["dj"]) for b in plan]
    assert sizes == [(0, 0, 60, 0), (0, 0, 60, 60), (0, 0, 10, 120),
                     (1, 200, 60, 0), (0, 200, 10, 60)]
    assert plan[0]["I"] == list(range(3, 63)) and plan[2]["I"] == list(range(123, 133))


def test_split_blocks_compose_to_recompute():
    """Consecutive Table 2 updates of one sink compose: Inc-bSR with a 60-source split and
    without it both reach the recompute of the updated graph at a deep series (the split
    only changes each part's truncation)."""
    n = 90
    s, d = W.chung_lu(n, 300, seed=741)
    es = set(zip(s.tolist(), d.tolist()))
    add = [(a, 5) for a in range(n) if a != 5 and (a, 5) not in es][:70]
    bi = [a for a, _ in add]
    bj = [b for _, b in add]
    S0 = O.fixed_point(Gr.transition_matrix(n, s, d), C)
    s2 = np.concatenate([s, bi])
    d2 = np.concatenate([d, bj])
    exact = O.fixed_point(Gr.transition_matrix(n, s2, d2), C)
    S1, plan = I.inc_bsr(n, s, d, S0, bi, bj, [1] * len(bi), C, 60, max_sources=60)
    assert [len(b["I"]) for b in plan] == [60, 10]
    assert np.abs(S1 - exact).max() < 1e-11
    S2, plan = I.inc_bsr(n, s, d, S0, bi, bj, [1] * len(bi), C, 60)
    assert [len(b["I"]) for b in plan] == [70]
    assert np.abs(S2 - exact).max() < 1e-11
