"""Pins of the oracle's affected-area sets (Theorem 4): soundness by brute force (the exact
Delta S vanishes outside A_hat x B_hat u B_hat x A_hat), and structural supports (computed
here by boolean path counting, independent of any floating point) giving the same sets as
the supports of the oracle's float S on insertion-only updates."""
import numpy as np

from oracle import graph as Gr
from oracle import incremental as I
from oracle import simrank as O

C = 0.6


def rand_graph(rng, n, p):
    e = [(a, b) for a in range(n) for b in range(n) if a != b and rng.random() < p]
    return (np.array([a for a, _ in e], dtype=np.int64),
            np.array([b for _, b in e], dtype=np.int64))


def structural_support(n, s, d):
    """S[a,b] != 0 iff a == b or some node reaches both a and b by walks of the same
    length k >= 1 (every term of eq (17) is nonnegative, so no cancellation):
    R = I; R <- R | (A R A^T > 0) with A[a, x] = 1 for an edge x -> a."""
    A = np.zeros((n, n), dtype=np.int64)
    A[np.asarray(d), np.asarray(s)] = 1
    R = np.eye(n, dtype=bool)
    for _ in range(n * n + 1):
        Rn = R | ((A @ R.astype(np.int64) @ A.T) > 0)
        if np.array_equal(Rn, R):
            break
        R = Rn
    return R


def test_aff_sound_random_updates():
    rng = np.random.default_rng(31)
    for trial in range(80):
        n = int(rng.integers(5, 11))
        s, d = rand_graph(rng, n, 0.25)
        Q = Gr.transition_matrix(n, s, d, dense=True)
        S = O.kron_solve(Q, C)
        es = set(zip(s.tolist(), d.tolist()))
        if trial % 2 == 0 or not es:
            absent = [(a, b) for a in range(n) for b in range(n) if a != b and (a, b) not in es]
            i, j = absent[int(rng.integers(len(absent)))]
            op = 1
        else:
            i, j = sorted(es)[int(rng.integers(len(es)))]
            op = -1
        n2, s2, d2 = Gr.apply_edges(n, s, d, [i], [j], [op])
        S2 = O.kron_solve(Gr.transition_matrix(n2, s2, d2, dense=True), C)
        for K in (0, 1, 3, 30):
            A, B, Ah, Bh = I.aff_for_update(n, s, d, S, [i], j, op, K, supp_eps=1e-13)
            mask = I.aff_pairs(Ah, Bh, n)
            # the K-truncated Delta S is supported inside the AFF
            deg = Gr.in_degrees(n, s, d)
            SK, info = I.inc_usr(Q, S, deg, i, j, C, K, op)
            assert np.abs((SK - S)[~mask]).max(initial=0.0) < 1e-15
            # each M_k lives on A_k x B_k u A_0 x B_0 (Theorem 4)
            Xi, H = info["Xi"], info["H"]
            Mk = np.zeros((n, n))
            for k in range(K + 1):
                Mk = Mk + np.outer(Xi[:, k], H[:, k])
                m = np.zeros((n, n), dtype=bool)
                m[np.ix_(A[k], B[k])] = True
                m[np.ix_(A[0], B[0])] = True
                assert np.abs(Mk[~m]).max(initial=0.0) < 1e-15
        # the exact Delta S as well (K = infinity)
        A, B, Ah, Bh = I.aff_for_update(n, s, d, S, [i], j, op, n + 1, supp_eps=1e-13)
        mask = I.aff_pairs(Ah, Bh, n)
        assert np.abs((S2 - S)[~mask]).max(initial=0.0) < 1e-13


def test_aff_float_support_equals_structural_on_insertions():
    import workloads as W
    n = 120
    s, d = W.chung_lu(n, 400, seed=41)
    i_s, j_s = W.insertion_stream(n, s, d, 6, seed=42)
    cur_s, cur_d = s.astype(np.int64), d.astype(np.int64)
    for i, j in zip(i_s.tolist(), j_s.tolist()):
        Q = Gr.transition_matrix(n, cur_s, cur_d)
        S = O.fixed_point(Q, C)
        R = structural_support(n, cur_s, cur_d)
        assert np.array_equal(S != 0.0, R)
        A1, B1, Ah1, Bh1 = I.aff_for_update(n, cur_s, cur_d, S, [i], j, 1, 15)
        # same sets from the structural support
        deg = Gr.in_degrees(n, cur_s, cur_d)
        out_old = Gr.out_neighbours(n, cur_s, cur_d)
        s2 = np.concatenate([cur_s, [i]])
        d2 = np.concatenate([cur_d, [j]])
        out_new = Gr.out_neighbours(n, s2, d2)
        supp_j = np.nonzero(R[j])[0] if deg[j] > 0 else None
        A2, B2, Ah2, Bh2 = I.aff_sets(out_old, out_new, np.nonzero(R[i])[0], supp_j, j, 15)
        assert all(np.array_equal(a, b) for a, b in zip(A1, A2))
        assert all(np.array_equal(a, b) for a, b in zip(B1, B2))
        cur_s, cur_d = s2, d2


def test_aff_pair_count_formula():
    rng = np.random.default_rng(5)
    for _ in range(20):
        n = 30
        Ah = np.unique(rng.integers(0, n, 12))
        Bh = np.unique(rng.integers(0, n, 17))
        assert I.aff_pair_count(Ah, Bh) == int(I.aff_pairs(Ah, Bh, n).sum())
