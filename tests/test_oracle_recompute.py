"""Pins of the oracle's SimRank recompute against things other than itself: the Kronecker
linear solve, closed forms (directed cycle, arborescence of the paper's Example 1.2,
isolated nodes, disjoint unions), and the invariants of eq (03a)."""
import numpy as np
import pytest

from oracle import graph as Gr
from oracle import simrank as O

C = 0.6


def rand_graph(rng, n, p):
    e = [(a, b) for a in range(n) for b in range(n) if a != b and rng.random() < p]
    return (np.array([a for a, _ in e], dtype=np.int64),
            np.array([b for _, b in e], dtype=np.int64))


def test_kron_equals_fixed_point_random():
    rng = np.random.default_rng(1)
    for _ in range(40):
        n = int(rng.integers(2, 10))
        s, d = rand_graph(rng, n, 0.35)
        Q = Gr.transition_matrix(n, s, d, dense=True)
        Sk = O.kron_solve(Q, C)
        Sf = O.fixed_point(Q, C)
        assert np.abs(Sk - Sf).max() < 1e-14
        # the fixed point satisfies eq (03a)
        assert np.abs(C * Q @ Sf @ Q.T + (1 - C) * np.eye(n) - Sf).max() < 1e-14


def test_kron_is_eq03a_directly():
    # vec form: solving eq (03a) entry by entry as a linear system built by hand
    rng = np.random.default_rng(2)
    n = 5
    s, d = rand_graph(rng, n, 0.4)
    Q = Gr.transition_matrix(n, s, d, dense=True)
    A = np.zeros((n * n, n * n))
    rhs = np.zeros(n * n)
    for a in range(n):
        for b in range(n):
            r = a * n + b
            A[r, r] += 1.0
            for x in range(n):
                for y in range(n):
                    A[r, x * n + y] -= C * Q[a, x] * Q[b, y]
            rhs[r] = (1 - C) if a == b else 0.0
    S = np.linalg.solve(A, rhs).reshape(n, n)
    assert np.abs(S - O.kron_solve(Q, C)).max() < 1e-14


def test_directed_cycle_is_identity():
    # Q is a permutation matrix, so S = I solves eq (03a): C P I P^T + (1-C) I = I
    for n in (3, 7, 40):
        s = np.arange(n)
        d = (s + 1) % n
        Q = Gr.transition_matrix(n, s, d)
        S = O.fixed_point(Q, C)
        assert np.abs(S - np.eye(n)).max() < 1e-14


def test_isolated_nodes():
    n = 6
    s = np.array([0, 1])
    d = np.array([1, 2])
    S = O.fixed_point(Gr.transition_matrix(n, s, d), C)
    for a in (3, 4, 5):   # no in- or out-edges
        row = np.zeros(n)
        row[a] = 1 - C
        assert np.abs(S[a] - row).max() < 1e-15
    # a root (no in-edges) has S_aa = 1 - C
    assert abs(S[0, 0] - (1 - C)) < 1e-15


def tree_closed_form(parent, C):
    """Example 1.2: S(a,b) = C^lam (1 - C^(H - lam + 1)) on the same level (H = depth,
    lam = edges from the lowest common ancestor to a), else 0."""
    n = len(parent)
    depth = np.zeros(n, dtype=int)
    for v in range(n):
        x, dep = v, 0
        while parent[x] >= 0:
            x = parent[x]
            dep += 1
        depth[v] = dep
    S = np.zeros((n, n))
    for a in range(n):
        for b in range(n):
            if depth[a] != depth[b]:
                continue
            x, y, lam = a, b, 0
            while x != y:
                x, y, lam = parent[x], parent[y], lam + 1
            H = depth[a]
            S[a, b] = C ** lam * (1 - C ** (H - lam + 1))
    return S


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_arborescence_closed_form(seed):
    rng = np.random.default_rng(seed)
    n = 30
    parent = [-1] + [int(rng.integers(v)) for v in range(1, n)]   # edges parent -> child
    s = np.array([parent[v] for v in range(1, n)])
    d = np.arange(1, n)
    for c in (0.6, 0.8):
        S = O.fixed_point(Gr.transition_matrix(n, s, d), c)
        assert np.abs(S - tree_closed_form(parent, c)).max() < 1e-14


def test_disjoint_union_block_diagonal():
    rng = np.random.default_rng(5)
    n1, n2 = 7, 6
    s1, d1 = rand_graph(rng, n1, 0.3)
    s2, d2 = rand_graph(rng, n2, 0.3)
    s = np.concatenate([s1, s2 + n1])
    d = np.concatenate([d1, d2 + n1])
    S = O.fixed_point(Gr.transition_matrix(n1 + n2, s, d), C)
    S1 = O.kron_solve(Gr.transition_matrix(n1, s1, d1), C)
    S2 = O.kron_solve(Gr.transition_matrix(n2, s2, d2), C)
    assert np.abs(S[:n1, :n1] - S1).max() < 1e-14
    assert np.abs(S[n1:, n1:] - S2).max() < 1e-14
    assert np.abs(S[:n1, n1:]).max() == 0.0


def test_invariants_chung_lu():
    import workloads as W
    s, d = W.chung_lu(300, 1500, seed=7)
    S = O.fixed_point(Gr.transition_matrix(300, s, d), C)
    assert np.abs(S - S.T).max() < 1e-14
    assert S.min() >= 0.0 and S.max() <= 1.0
    assert np.diag(S).min() >= 1 - C - 1e-15


def test_partial_sim_equals_truncated_series():
    rng = np.random.default_rng(3)
    n = 25
    s, d = rand_graph(rng, n, 0.12)
    Q = Gr.transition_matrix(n, s, d)
    for K in (0, 1, 5, 12):
        T = O.truncated(Q, C, K)
        for q in range(n):
            assert np.abs(O.partial_sim(Q, q, K, C) - T[:, q]).max() < 1e-15
    # the K-term series is the K-th fixed-point iterate from (1 - C) I
    Qd = Q.toarray()
    S = (1 - C) * np.eye(n)
    for _ in range(6):
        S = C * Qd @ S @ Qd.T + (1 - C) * np.eye(n)
    assert np.abs(S - O.truncated(Q, C, 6)).max() < 1e-15


def test_single_source_tail_bound():
    import workloads as W
    s, d = W.chung_lu(400, 2400, seed=9)
    Q = Gr.transition_matrix(400, s, d)
    S = O.fixed_point(Q, C)
    for q in (0, 5, 17, 399):
        assert np.abs(O.single_source(Q, q, C, tol=1e-13) - S[:, q]).max() < 1e-13
    # a shallow PartialSim misses by at most C^(K+1)
    for K in (3, 6, 10):
        err = max(np.abs(O.partial_sim(Q, q, K, C) - S[:, q]).max() for q in (0, 5, 17))
        assert err <= C ** (K + 1)
