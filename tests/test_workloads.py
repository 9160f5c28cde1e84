"""The seeded generators: determinism, simple-digraph properties, valid update streams."""
import numpy as np
import pytest

import workloads as W


def test_chung_lu_simple_and_deterministic():
    s, d = W.chung_lu(1000, 5000, seed=1001)
    assert len(s) == 5000
    assert (s != d).all()
    assert len(set(zip(s.tolist(), d.tolist()))) == 5000
    s2, d2 = W.chung_lu(1000, 5000, seed=1001)
    assert np.array_equal(s, s2) and np.array_equal(d, d2)
    deg = np.bincount(d, minlength=1000)
    assert deg.max() > 50          # power-law hubs
    assert (deg == 0).mean() > 0.05


def test_streams_are_valid():
    s, d = W.chung_lu(500, 2500, seed=3)
    es = set(zip(s.tolist(), d.tolist()))
    i, j, o = W.mixed_stream(500, s, d, 300, 0.7, 4)
    for a, b, op in zip(i.tolist(), j.tolist(), o.tolist()):
        assert a != b
        if op > 0:
            assert (a, b) not in es
            es.add((a, b))
        else:
            assert (a, b) in es
            es.remove((a, b))
    assert 0.55 < (o > 0).mean() < 0.85


def test_batch_stream_new_ids_dense():
    s, d = W.chung_lu(400, 2000, seed=5)
    batches, counts = W.batch_stream(400, s, d, 4, 200, 6)
    cur = 400
    for (i, j, o), nn in zip(batches, counts):
        ids = sorted({x for x in np.concatenate([i, j]).tolist() if x >= cur})
        assert ids == list(range(cur, nn))
        cur = nn


def test_loss_pairs_unique():
    a, b, t = W.loss_pairs(100, 500, 7)
    assert (a < b).all()
    assert len(set(zip(a.tolist(), b.tolist()))) == 500
    assert (t >= 0).all() and (t < 0.2).all()


def test_with_hubs_exact_degrees():
    n = 3000
    s, d = W.chung_lu(n, 9000, seed=91)
    s2, d2 = W.with_hubs(n, s, d, [(3, 2500, 1200), (4, 700, 10)], seed=92)
    assert np.array_equal(s2[:len(s)], s) and np.array_equal(d2[:len(d)], d)
    assert len(set(zip(s2.tolist(), d2.tolist()))) == len(s2)
    assert np.all(s2 != d2)
    ind = np.bincount(d2, minlength=n)
    outd = np.bincount(s2, minlength=n)
    assert (ind[3], outd[3], ind[4], outd[4]) == (2500, 1200, 700, 10)
    s3, d3 = W.with_hubs(n, s, d, [(3, 2500, 1200), (4, 700, 10)], seed=92)
    assert np.array_equal(s2, s3) and np.array_equal(d2, d3)
    with pytest.raises(ValueError):
        W.with_hubs(n, s2, d2, [(3, 10, 10)], seed=93)


def test_existing_batch_valid():
    n = 500
    s, d = W.chung_lu(n, 2500, seed=95)
    bi, bj, bo = W.existing_batch(n, s, d, n_ins=12, n_del=5, shared=4, seed=96)
    es = set(zip(s.tolist(), d.tolist()))
    ins = [(a, b) for a, b, o in zip(bi.tolist(), bj.tolist(), bo.tolist()) if o > 0]
    dels = [(a, b) for a, b, o in zip(bi.tolist(), bj.tolist(), bo.tolist()) if o < 0]
    assert len(ins) == 12 and len(dels) == 5
    assert len(set(ins)) == 12 and not (set(ins) & es) and all(a != b for a, b in ins)
    assert len(set(dels)) == 5 and set(dels) <= es
    assert len({b for _, b in ins[:4]}) == 1
    assert np.all(bi < n) and np.all(bj < n)
    b2 = W.existing_batch(n, s, d, n_ins=12, n_del=5, shared=4, seed=96)
    assert all(np.array_equal(x, y) for x, y in zip((bi, bj, bo), b2))


def test_existing_batches_apply_in_sequence():
    n = 400
    s, d = W.chung_lu(n, 2000, seed=97)
    batches = W.existing_batches(n, s, d, 3, n_ins=10, n_del=4, shared=3, seed=98)
    assert len(batches) == 3
    cur = set(zip(s.tolist(), d.tolist()))
    for bi, bj, bo in batches:
        assert len(bi) == 14 and bo.tolist() == [1] * 10 + [-1] * 4
        ins = list(zip(bi[:10].tolist(), bj[:10].tolist()))
        dels = list(zip(bi[10:].tolist(), bj[10:].tolist()))
        assert len({b for _, b in ins[:3]}) == 1
        assert not (set(ins) & cur) and set(dels) <= cur
        cur |= set(ins)
        cur -= set(dels)
    one = W.existing_batches(n, s, d, 1, n_ins=10, n_del=4, shared=3, seed=98)[0]
    assert all(np.array_equal(x, y)
               for x, y in zip(one, W.existing_batch(n, s, d, 10, 4, 3, seed=98)))


def test_communities_planted_groups():
    n, m, parts = 1000, 6000, 5
    s, d, g = W.communities(n, m, parts, 0.03, seed=99)
    assert len(s) == m and len(set(zip(s.tolist(), d.tolist()))) == m and np.all(s != d)
    assert np.bincount(g).tolist() == [200] * 5
    assert (g[s] != g[d]).sum() == 180
    s2, d2, g2 = W.communities(n, m, parts, 0.03, seed=99)
    assert np.array_equal(s, s2) and np.array_equal(d, d2) and np.array_equal(g, g2)
