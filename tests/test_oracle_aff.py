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


def test_xi_lives_on_the_sinks_k_step_out_walks():
    """xi_0 = C e_j and xi_{k+1} = C Qt xi_k with Qt = Q + u v^T the new graph's transition
    matrix, so xi_k is zero outside W_k, the nodes reached from the sink j by a walk of exactly
    k out-steps in the new graph (W_0 = {j}, W_{k+1} = out_new(W_k)), computed here by boolean
    steps on the edge list. The fused pass's tile skipping rests on this sparsity. The series
    run on the new graph's Q (as the device runs it) is supported on W_k exactly and equals the
    oracle's series; the oracle's own form, old Q plus the rank-one term, is too on insertions,
    while on deletions the deleted edge's term in row j cancels only to rounding, leaving
    residues below 1e-15 of the vector's size that walk on from j. Insertion and deletion
    blocks on random graphs; on insertions the first steps fill W_k (all terms nonnegative)."""
    rng = np.random.default_rng(2024)
    K = 6
    for trial in range(30):
        n = int(rng.integers(12, 40))
        s, d = rand_graph(rng, n, 0.12)
        if len(s) < 3:
            continue
        es = set(zip(s.tolist(), d.tolist()))
        op = 1 if trial % 2 == 0 else -1
        if op > 0:
            j = int(rng.integers(n))
            cand = [i for i in range(n) if i != j and (i, j) not in es]
            I_ = sorted(rng.choice(cand, size=min(3, len(cand)), replace=False).tolist())
        else:
            j = int(d[rng.integers(len(d))])
            srcs = sorted(int(a) for a, b in es if b == j)
            I_ = srcs[:max(1, len(srcs) // 2)]
        Q = Gr.transition_matrix(n, s, d)
        deg = np.bincount(d, minlength=n)
        S = O.fixed_point(Q, C)
        _, info = I.inc_block(Q, S, deg, I_, j, C, K, op)
        new = es | {(i, j) for i in I_} if op > 0 else es - {(i, j) for i in I_}
        out = [[] for _ in range(n)]
        for a, b in new:
            out[a].append(b)
        ns, nd = zip(*sorted(new)) if new else ((), ())
        Qn = Gr.transition_matrix(n, np.asarray(ns, np.int64), np.asarray(nd, np.int64))
        xn = np.zeros(n)
        xn[j] = C
        W = {j}
        for k in range(K + 1):
            Xi = info["Xi"][:, k]
            scale = max(float(np.max(np.abs(Xi))), 1e-300)
            nz = set(np.nonzero(xn)[0].tolist())
            assert nz <= W, (trial, k, sorted(nz - W))
            assert np.max(np.abs(xn - Xi)) <= 1e-12 * scale, (trial, k)
            out_w = np.ones(n, dtype=bool)
            out_w[list(W)] = False
            if op > 0:
                assert not np.any(Xi[out_w]), (trial, k)
                if k <= 2:
                    assert nz == W, (trial, k)
            else:
                assert np.max(np.abs(Xi[out_w]), initial=0.0) <= 1e-15 * scale, (trial, k)
            W = {b for a in W for b in out[a]}
            xn = C * (Qn @ xn)
