"""Pins of the oracle's incremental formulas: brute force (Kronecker solve on the updated
graph) over every 4-node digraph and every single-edge update, random small graphs for
Table 2 blocks and node insertions, the delta = 1 reduction, the truncation bound, and the
arithmetic of the paper's worked examples (tests/golden/worked_examples.json)."""
import json
import os

import numpy as np
import pytest

from oracle import graph as Gr
from oracle import incremental as I
from oracle import simrank as O

C = 0.6
HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "worked_examples.json")))


def rand_graph(rng, n, p):
    e = [(a, b) for a in range(n) for b in range(n) if a != b and rng.random() < p]
    return (np.array([a for a, _ in e], dtype=np.int64),
            np.array([b for _, b in e], dtype=np.int64))


def exact_after(n, s, d, ui, uj, uop, n_new=None):
    n2, s2, d2 = Gr.apply_edges(n, s, d, ui, uj, uop, n_new=n_new)
    return O.kron_solve(Gr.transition_matrix(n2, s2, d2, dense=True), C)


def test_exhaustive_four_node_single_edge_updates():
    """Every labelled digraph on 4 nodes (2^12) and every single-edge insertion or deletion,
    closed form (Theorems 3/9) at K = 70: the incremental S equals the Kronecker solve."""
    n = 4
    pairs = [(a, b) for a in range(n) for b in range(n) if a != b]
    worst = 0.0
    count = 0
    for mask in range(1 << len(pairs)):
        e = [pairs[t] for t in range(len(pairs)) if mask >> t & 1]
        s = np.array([a for a, _ in e], dtype=np.int64)
        d = np.array([b for _, b in e], dtype=np.int64)
        Q = Gr.transition_matrix(n, s, d, dense=True)
        S = O.kron_solve(Q, C)
        deg = Gr.in_degrees(n, s, d)
        # one insertion and one deletion per graph, chosen by the mask
        absent = [p for p in pairs if p not in e]
        for (ops, pool) in ((1, absent), (-1, e)):
            if not pool:
                continue
            i, j = pool[mask % len(pool)]
            Sn, _ = I.inc_usr(Q, S, deg, i, j, C, 70, ops, "closed")
            worst = max(worst, np.abs(Sn - exact_after(n, s, d, [i], [j], [ops])).max())
            count += 1
    assert count > 8000
    assert worst < 5e-15


@pytest.mark.parametrize("form", ["closed", "direct"])
def test_unit_updates_random(form):
    rng = np.random.default_rng(11)
    for _ in range(60):
        n = int(rng.integers(5, 11))
        s, d = rand_graph(rng, n, 0.3)
        Q = Gr.transition_matrix(n, s, d, dense=True)
        S = O.kron_solve(Q, C)
        deg = Gr.in_degrees(n, s, d)
        es = set(zip(s.tolist(), d.tolist()))
        absent = [(a, b) for a in range(n) for b in range(n) if a != b and (a, b) not in es]
        i, j = absent[int(rng.integers(len(absent)))]
        Sn, _ = I.inc_usr(Q, S, deg, i, j, C, 80, 1, form)
        assert np.abs(Sn - exact_after(n, s, d, [i], [j], [1])).max() < 1e-14
        if es:
            i, j = sorted(es)[int(rng.integers(len(es)))]
            Sn, _ = I.inc_usr(Q, S, deg, i, j, C, 80, -1, form)
            assert np.abs(Sn - exact_after(n, s, d, [i], [j], [-1])).max() < 1e-14


def test_rank_one_factors_reproduce_new_Q():
    rng = np.random.default_rng(12)
    for _ in range(40):
        n = 8
        s, d = rand_graph(rng, n, 0.3)
        Q = Gr.transition_matrix(n, s, d, dense=True)
        deg = Gr.in_degrees(n, s, d)
        es = set(zip(s.tolist(), d.tolist()))
        absent = [(a, b) for a in range(n) for b in range(n) if a != b and (a, b) not in es]
        i, j = absent[0]
        u, v = I.rank_one_insert(Q, deg, i, j)
        n2, s2, d2 = Gr.apply_edges(n, s, d, [i], [j], [1])
        assert np.abs(Q + np.outer(u, v) - Gr.transition_matrix(n2, s2, d2, dense=True)).max() < 1e-15
        if es:
            i, j = sorted(es)[0]
            u, v = I.rank_one_delete(Q, deg, i, j)
            n2, s2, d2 = Gr.apply_edges(n, s, d, [i], [j], [-1])
            assert np.abs(Q + np.outer(u, v) - Gr.transition_matrix(n2, s2, d2, dense=True)).max() < 1e-15


@pytest.mark.parametrize("form", ["closed", "direct"])
def test_table2_c0_blocks(form):
    rng = np.random.default_rng(13)
    for _ in range(50):
        n = int(rng.integers(5, 10))
        s, d = rand_graph(rng, n, 0.35)
        Q = Gr.transition_matrix(n, s, d, dense=True)
        S = O.kron_solve(Q, C)
        deg = Gr.in_degrees(n, s, d)
        es = set(zip(s.tolist(), d.tolist()))
        j = int(rng.integers(n))
        cand = [a for a in range(n) if a != j and (a, j) not in es]
        if cand:
            Ib = sorted(rng.choice(cand, size=int(rng.integers(1, len(cand) + 1)), replace=False).tolist())
            Sn, _ = I.inc_block(Q, S, deg, Ib, j, C, 80, 1, form)
            assert np.abs(Sn - exact_after(n, s, d, Ib, [j] * len(Ib), [1] * len(Ib))).max() < 1e-14
            u, v = I.rank_one_block(Q, deg, Ib, j, 1)
            n2, s2, d2 = Gr.apply_edges(n, s, d, Ib, [j] * len(Ib), [1] * len(Ib))
            assert np.abs(Q + np.outer(u, v) - Gr.transition_matrix(n2, s2, d2, dense=True)).max() < 1e-15
        ins = [a for (a, b) in es if b == j]
        if ins:
            Ib = sorted(rng.choice(ins, size=int(rng.integers(1, len(ins) + 1)), replace=False).tolist())
            Sn, _ = I.inc_block(Q, S, deg, Ib, j, C, 80, -1, form)
            assert np.abs(Sn - exact_after(n, s, d, Ib, [j] * len(Ib), [-1] * len(Ib))).max() < 1e-14


def test_delta_one_reduces_to_unit_theorems():
    rng = np.random.default_rng(14)
    for _ in range(30):
        n = 9
        s, d = rand_graph(rng, n, 0.3)
        Q = Gr.transition_matrix(n, s, d, dense=True)
        S = O.kron_solve(Q, C)
        deg = Gr.in_degrees(n, s, d)
        es = set(zip(s.tolist(), d.tolist()))
        absent = [(a, b) for a in range(n) for b in range(n) if a != b and (a, b) not in es]
        i, j = absent[int(rng.integers(len(absent)))]
        u1, v1 = I.rank_one_insert(Q, deg, i, j)
        ub, vb = I.rank_one_block(Q, deg, [i], j, 1)
        assert np.array_equal(u1, ub) and np.abs(v1 - vb).max() < 1e-16
        g1 = I.gamma_closed(Q, S, deg, [i], j, C, 1)
        # Theorem 3 typed in its unit form (eq (29aa)/(29bb)/(29b)) against the block form
        QSi = Q @ S[:, i]
        lam = S[i, i] + S[j, j] / C - 2 * Q[j, :] @ S[:, i] - 1 / C + 1
        ej = np.eye(n)[j]
        if deg[j] == 0:
            g_unit = QSi + 0.5 * S[i, i] * ej
        else:
            g_unit = (QSi - S[:, j] / C + (lam / (2 * (deg[j] + 1)) + 1 / C - 1) * ej) / (deg[j] + 1)
        assert np.abs(g1 - g_unit).max() < 1e-15


def test_node_insertion_cases():
    rng = np.random.default_rng(15)
    for _ in range(40):
        n = int(rng.integers(4, 9))
        s, d = rand_graph(rng, n, 0.3)
        Q = Gr.transition_matrix(n, s, d, dense=True)
        S = O.kron_solve(Q, C)
        deg = Gr.in_degrees(n, s, d)
        delta = int(rng.integers(1, 4))
        Iset = sorted(rng.choice(n, size=min(delta, n), replace=False).tolist())
        # C1: existing sources I -> new sink n (Theorem 8 / Table 2)
        got = I.c1_block(Q, S, Iset, C)
        assert np.abs(got - exact_after(n, s, d, Iset, [n] * len(Iset), [1] * len(Iset))).max() < 1e-14
        # C2: new sources n..n+delta-1 -> existing sink j (Theorems 5-7 / Table 2)
        j = int(rng.integers(n))
        got, _ = I.c2_block(Q, S, deg, delta, j, C, 80)
        exp = exact_after(n, s, d, list(range(n, n + delta)), [j] * delta, [1] * delta)
        assert np.abs(got - exp).max() < 1e-14
        # C3: new sources -> new sink (Algorithm 5 / Table 2)
        got = I.c3_block(S, delta, C)
        exp = exact_after(n, s, d, list(range(n, n + delta)), [n + delta] * delta, [1] * delta)
        assert np.abs(got - exp).max() < 1e-15


def test_c3_closed_form_values():
    S = I.c3_block(np.zeros((0, 0)), 1, C)
    assert np.abs(S - np.diag([1 - C, 1 - C * C])).max() <= 2.3e-16   # (1-C)(1+C) = 1-C^2
    S = I.c3_block(np.zeros((0, 0)), 4, C)
    assert abs(S[4, 4] - (1 - C) * (1 + C / 4)) == 0.0


def test_c2_equals_isolated_node_then_c0():
    """A new source is an isolated node (S entry 1 - C on its diagonal) until its edge
    arrives, so C2 equals "add isolated nodes, then the Table 2 (C0) insert block"."""
    rng = np.random.default_rng(16)
    for _ in range(30):
        n = int(rng.integers(4, 9))
        s, d = rand_graph(rng, n, 0.35)
        Q = Gr.transition_matrix(n, s, d, dense=True)
        S = O.kron_solve(Q, C)
        deg = Gr.in_degrees(n, s, d)
        delta = int(rng.integers(1, 4))
        j = int(rng.integers(n))
        c2, _ = I.c2_block(Q, S, deg, delta, j, C, 60)
        Sg = I.grow(S, delta)
        for t in range(delta):
            Sg[n + t, n + t] = 1 - C
        Qg = np.zeros((n + delta, n + delta))
        Qg[:n, :n] = Q
        degg = np.concatenate([deg, np.zeros(delta, dtype=deg.dtype)])
        viaC0, _ = I.inc_block(Qg, Sg, degg, list(range(n, n + delta)), j, C, 60, 1)
        assert np.abs(c2 - viaC0).max() < 1e-15


def test_truncation_bound_holds():
    import workloads as W
    n = 200
    s, d = W.chung_lu(n, 1000, seed=21)
    Q = Gr.transition_matrix(n, s, d, dense=True)
    S = O.fixed_point(Gr.transition_matrix(n, s, d), C)
    deg = Gr.in_degrees(n, s, d)
    es = set(zip(s.tolist(), d.tolist()))
    rng = np.random.default_rng(3)
    for _ in range(6):
        while True:
            i, j = int(rng.integers(n)), int(rng.integers(n))
            if i != j and (i, j) not in es:
                break
        S_inf, info = I.inc_usr(Q, S, deg, i, j, C, 90, 1)
        u, v = info["u"], info["v"]
        w = I.w_direct(Q, S, u, v)
        for K in (5, 10, 15):
            S_K, _ = I.inc_usr(Q, S, deg, i, j, C, K, 1)
            err = np.abs(S_K - S_inf).max()
            assert err <= I.truncation_bound(C, K, u, w) * (1 + 1e-9) + 1e-16


# ----------------------------------------------------------------------------- worked examples

def test_worked_example_inc_usr_gamma():
    g = GOLD["inc_usr_example"]
    c = g["C"]
    names = ["a", "b", "f", "i", "j"]
    idx = {x: p for p, x in enumerate(names)}
    n = len(names)
    QSi = np.zeros(n)
    QSi[idx["a"]] = g["w"]["a"]
    QSi[idx["b"]] = g["w"]["b"]
    QSi[idx["j"]] = g["w_j"]
    Sj = np.zeros(n)
    for k, val in g["S_col_j"].items():
        Sj[idx[k]] = val
    lam = g["S_ii"] + g["S_jj"] / c - 2 * g["w_j"] - 1 / c + 1     # eq (29b)
    assert abs(lam - g["lambda"]) < 5e-4
    gamma = I.gamma_closed_parts(QSi, Sj, g["S_ii"], g["S_jj"], g["d_j"], 1, idx["j"], c, 1)
    for k, val in g["gamma"].items():
        assert abs(gamma[idx[k]] - val) < g["tol"], (k, gamma[idx[k]], val)


def test_worked_example_thm1():
    g = GOLD["thm1_example"]
    names = ["h", "i", "j", "k"]
    idx = {x: p for p, x in enumerate(names)}
    Q = np.zeros((4, 4))
    for k, val in g["Q_row_j"].items():
        Q[idx["j"], idx[k]] = val
    u, v = I.rank_one_insert(Q, np.array([0, 0, g["d_j"], 0]), idx["i"], idx["j"])
    assert abs(u[idx["j"]] - g["u_j"]) < 1e-15
    for k, val in g["v"].items():
        assert v[idx[k]] == val


def test_worked_example_c1():
    g = GOLD["c1_example"]
    c = g["C"]
    assert abs(c * g["S_ii"] + 1 - c - g["z"]) < 1e-4        # corner of eq (62)
    w = GOLD["inc_usr_example"]["w"]                          # Q S[:, i], same graph
    for k in ("a", "b"):
        assert abs(c * w[k] - g["y"][k]) < g["tol"]


def test_worked_example_c2():
    g = GOLD["c2_example"]
    c = g["C"]
    names = ["f", "i", "j"]
    idx = {x: p for p, x in enumerate(names)}
    Sj = np.array([g["S_col_j"][x] for x in names])
    z = I.c2_z(Sj, g["S_col_j"]["j"], g["d_j"], 1, idx["j"], c)
    for k, val in g["z"].items():
        assert abs(z[idx[k]] - val) < g["tol"]
    # k = 0 term of eq (59) scaled by C / (d_j + 1)
    ej = np.eye(3)[idx["j"]]
    dS0 = c / (g["d_j"] + 1) * (np.outer(ej, z) + np.outer(z, ej))
    for k, val in g["dS11_col_j"].items():
        assert abs(dS0[idx[k], idx["j"]] - val) < g["tol"]


def test_worked_example_aff_union_rectangle():
    """Theorem 4 example: with A_0 = {j}, B_0 = {a,b,f,i,j}, A_1 = {a,b}, B_1 = {a,b,d,j},
    M_1 is computed on (A_0 u A_1) x (B_0 u B_1), 3 x 6 = 18 entries. A graph whose
    out-neighbourhoods give those sets reproduces them through ``aff_sets``."""
    g = GOLD["aff_example"]
    names = ["a", "b", "c", "d", "e", "f", "i", "j", "x"]
    idx = {x: p for p, x in enumerate(names)}
    # out-edges chosen so that O(j) = {a, b} and O({a,b,f,i,j}) = {a, b, d, j}, and F1 comes
    # from supp S[i,:] = {x} with O(x) = {a, b}
    edges = [("j", "a"), ("j", "b"), ("a", "d"), ("b", "a"), ("f", "j"), ("i", "b"),
             ("x", "a"), ("x", "b")]
    n = len(names)
    s = [idx[a] for a, _ in edges]
    t = [idx[b] for _, b in edges]
    out = Gr.out_neighbours(n, s, t)
    A, B, Ah, Bh = I.aff_sets(out, out, [idx["x"]], [idx[v] for v in g["F2"]], idx["j"], 1)
    nm = lambda arr: sorted(names[v] for v in arr)
    assert nm(A[0]) == g["A0"] and nm(B[0]) == g["B0"]
    assert nm(A[1]) == g["A1"] and nm(B[1]) == g["B1"]
    rect = (sorted(set(nm(A[0])) | set(nm(A[1]))), sorted(set(nm(B[0])) | set(nm(B[1]))))
    assert [rect[0], rect[1]] == g["M1_rect"]
    assert len(rect[0]) * len(rect[1]) == g["M1_entries"]
