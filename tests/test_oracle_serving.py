"""Pins of the oracle's top-k selection: a worked example with ties, brute force by Python
sorting on random vectors with many ties, and precision@k on hand lists."""
import numpy as np

from oracle import serving as Sv


def test_worked_example_with_ties():
    col = [0.2, 0.5, 0.1, 0.5, 1.0, 0.2, 0.0]
    ids, vals = Sv.topk(col, 4, 4)          # query 4 (the largest) is left out
    assert ids.tolist() == [1, 3, 0, 5] and vals.tolist() == [0.5, 0.5, 0.2, 0.2]
    ids, vals = Sv.topk(col, 4, 3, exclude_self=False)
    assert ids.tolist() == [4, 1, 3]
    ids, _ = Sv.topk(col, 0, 7, exclude_self=False)
    assert ids.tolist() == [4, 1, 3, 0, 5, 2, 6]


def test_brute_force_on_random_vectors_with_ties():
    g = np.random.default_rng(5)
    for _ in range(50):
        n = int(g.integers(1, 300))
        col = np.round(g.random(n), 1) * (g.random(n) < 0.7)    # many equal values and zeros
        x = int(g.integers(n))
        k = int(g.integers(1, n + 1))
        for ex in (True, False):
            cand = [(-col[b], b) for b in range(n) if not (ex and b == x)]
            want = sorted(cand)[:k]
            ids, vals = Sv.topk(col, x, k, exclude_self=ex)
            assert ids.tolist() == [b for _, b in want]
            assert vals.tolist() == [-v for v, _ in want]


def test_precision_at_k():
    assert Sv.precision_at_k([1, 2, 3], [3, 2, 1]) == 1.0
    assert Sv.precision_at_k([1, 2, 9], [1, 2, 3]) == 2 / 3
    assert Sv.precision_at_k([], [1]) == 0.0
