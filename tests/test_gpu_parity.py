"""GPU parity: the HIP path through the C ABI against the oracle, on seeded Chung-Lu graphs.

Bars: AFF sets and batch plans bit-exact; S within 1e-6 max-abs of the oracle's converged
recompute of the updated graph (plus the rigorous truncation bound where it is tighter)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import adjoint as OA
from oracle import graph as Gr
from oracle import incremental as OI
from oracle import simrank as O

from _util import EdgeTracker, maxabs

pytestmark = pytest.mark.gpu

C = 0.6
TOL = 1e-6


def ctx_for(n, s, d, **kw):
    from paper_1711_00121_amd import Context
    return Context(n, s, d, **kw)


def test_mfma_f64_lane_layout():
    """v_mfma_f64_16x16x4_f64: lane l supplies A[l%16][l//16] and B[l//16][l%16]; slot v of
    lane l holds D[4*v + l//16][l%16]. The update kernel relies on this layout."""
    from paper_1711_00121_amd import mfma_layout_probe
    a = torch.arange(64, dtype=torch.float64) * 0.5 + 1.0
    b = torch.arange(64, dtype=torch.float64) * 0.25 - 3.0
    out = mfma_layout_probe(a, b).cpu().numpy()
    A = np.zeros((16, 4))
    B = np.zeros((4, 16))
    for l in range(64):
        A[l % 16, l // 16] = a[l]
        B[l // 16, l % 16] = b[l]
    D = A @ B
    exp = np.zeros(256)
    for l in range(64):
        for v in range(4):
            exp[4 * l + v] = D[4 * v + l // 16, l % 16]
    assert np.array_equal(out, exp)


def test_init_matches_oracle_fixed_point():
    n = 400
    s, d = W.chung_lu(n, 2000, seed=11)
    ctx = ctx_for(n, s, d, s_prec="fp64")
    S = ctx.S().cpu().numpy()
    Sx = O.fixed_point(Gr.transition_matrix(n, s, d), C)
    assert maxabs(S, Sx) < 1e-13


def test_c0_insertions_fp64_workload1_shape():
    """Workload 1 (n=1000, m=5000, K=15, FP64), 20 insertions, parity after every update and
    the rigorous truncation bound accumulated over the stream."""
    cfg = W.WORKLOADS[1]
    n = cfg["n"]
    s, d = W.chung_lu(n, cfg["m"], seed=1001)
    ii, jj = W.insertion_stream(n, s, d, cfg["updates"], seed=2001)
    ctx = ctx_for(n, s, d, s_prec="fp64", K=cfg["K"], C=cfg["C"])
    tr = EdgeTracker(n, s, d)
    bound = 0.0
    worst = 0.0
    for i, j in zip(ii.tolist(), jj.tolist()):
        st = ctx.apply_edge_update(i, j, 1, stats=True)
        tr.apply(i, j, 1)
        bound += st["bound"]
        err = maxabs(ctx.S().cpu().numpy(), tr.exact(C))
        worst = max(worst, err)
        assert err < TOL, (i, j, err)
        assert err <= bound + 1e-9
        assert st["pairs"] == 2 * st["aff_A"] * st["aff_B"] - st["aff_AB"] ** 2
    print(f"workload-1 shape: max |S_gpu - S*| = {worst:.3e}, accumulated bound {bound:.3e}")


@pytest.mark.parametrize("form", ["closed", "direct"])
@pytest.mark.parametrize("prune", [True, False])
def test_mixed_stream_fp64(form, prune):
    n = 500
    s, d = W.chung_lu(n, 3000, seed=21)
    ii, jj, oo = W.mixed_stream(n, s, d, 40, 0.7, seed=22)
    ctx = ctx_for(n, s, d, s_prec="fp64", gamma_form=form, prune=prune)
    tr = EdgeTracker(n, s, d)
    for t, (i, j, o) in enumerate(zip(ii.tolist(), jj.tolist(), oo.tolist())):
        ctx.apply_edge_update(i, j, o)
        tr.apply(i, j, o)
        if t in (0, 9, 39):
            assert maxabs(ctx.S().cpu().numpy(), tr.exact(C)) < TOL


@pytest.mark.parametrize("prec", ["hilo", "fp32"])
def test_float32_stores(prec):
    n = 500
    s, d = W.chung_lu(n, 3000, seed=31)
    ii, jj, oo = W.mixed_stream(n, s, d, 60, 0.7, seed=32)
    c64 = ctx_for(n, s, d, s_prec="fp64")
    c32 = ctx_for(n, s, d, s_prec=prec)
    tr = EdgeTracker(n, s, d)
    for i, j, o in zip(ii.tolist(), jj.tolist(), oo.tolist()):
        c64.apply_edge_update(i, j, o)
        c32.apply_edge_update(i, j, o)
        tr.apply(i, j, o)
    S64 = c64.S().cpu().numpy()
    S32 = c32.S().cpu().numpy()
    exact = tr.exact(C)
    d32 = maxabs(S32, S64)
    print(f"{prec}: max |S_{prec} - S_fp64| = {d32:.3e}, vs oracle {maxabs(S32, exact):.3e}")
    if prec == "hilo":
        assert d32 < 1e-9
        assert maxabs(S32, exact) < TOL
    else:
        assert d32 < 1e-5


def test_aff_sets_bit_exact_on_insertions():
    """Insert-only updates: the S supports are structural on both sides, so the GPU sets
    A_0..A_K, B_0..B_K and their unions equal the oracle's, element for element."""
    n = 300
    K = 15
    s, d = W.chung_lu(n, 1000, seed=41)
    ii, jj = W.insertion_stream(n, s, d, 6, seed=42)
    ctx = ctx_for(n, s, d, s_prec="fp64", K=K)
    cur_s, cur_d = s.astype(np.int64), d.astype(np.int64)
    for i, j in zip(ii.tolist(), jj.tolist()):
        S_or = O.fixed_point(Gr.transition_matrix(n, cur_s, cur_d), C)
        A, B, Ah, Bh = OI.aff_for_update(n, cur_s, cur_d, S_or, [i], j, 1, K)
        ctx.apply_edge_update(i, j, 1)
        for lvl in range(K + 1):
            ga, gb = ctx.get_aff(lvl)
            assert np.array_equal(ga.cpu().numpy(), A[lvl]), ("A", lvl)
            assert np.array_equal(gb.cpu().numpy(), B[lvl]), ("B", lvl)
        ga, gb = ctx.get_aff(-1)
        assert np.array_equal(ga.cpu().numpy(), Ah)
        assert np.array_equal(gb.cpu().numpy(), Bh)
        cur_s = np.concatenate([cur_s, [i]])
        cur_d = np.concatenate([cur_d, [j]])


def test_aff_sets_bit_exact_mid_size():
    """The affected areas at n = 2000 over several tiles of the compaction and traversal
    kernels (light, medium and heavy rows), against the oracle's sets from the exact S."""
    n = 2000
    K = 15
    s, d = W.chung_lu(n, 16000, seed=141)
    ii, jj = W.insertion_stream(n, s, d, 3, seed=142)
    ctx = ctx_for(n, s, d, s_prec="fp64", K=K)
    cur_s, cur_d = s.astype(np.int64), d.astype(np.int64)
    for i, j in zip(ii.tolist(), jj.tolist()):
        S_or = O.fixed_point(Gr.transition_matrix(n, cur_s, cur_d), C)
        A, B, Ah, Bh = OI.aff_for_update(n, cur_s, cur_d, S_or, [i], j, 1, K)
        ctx.apply_edge_update(i, j, 1)
        for lvl in (0, 1, 2, K):
            ga, gb = ctx.get_aff(lvl)
            assert np.array_equal(ga.cpu().numpy(), A[lvl]), ("A", lvl)
            assert np.array_equal(gb.cpu().numpy(), B[lvl]), ("B", lvl)
        ga, gb = ctx.get_aff(-1)
        assert np.array_equal(ga.cpu().numpy(), Ah)
        assert np.array_equal(gb.cpu().numpy(), Bh)
        cur_s = np.append(cur_s, i)
        cur_d = np.append(cur_d, j)
    # deletions, each as the first update of a fresh context (its S is the converged one, so
    # both sides take supports from the same S): an edge into a sink with several in-edges,
    # and the only in-edge of a sink (F2 empty)
    S_or = O.fixed_point(Gr.transition_matrix(n, s, d), C)
    indeg = np.bincount(d, minlength=n)
    e_multi = int(np.nonzero(indeg[d] > 1)[0][0])
    e_single = int(np.nonzero(indeg[d] == 1)[0][0])
    for e in (e_multi, e_single):
        i, j = int(s[e]), int(d[e])
        A, B, Ah, Bh = OI.aff_for_update(n, s.astype(np.int64), d.astype(np.int64), S_or, [i],
                                         j, -1, K)
        ctx = ctx_for(n, s, d, s_prec="fp64", K=K)
        ctx.apply_edge_update(i, j, -1)
        ga, gb = ctx.get_aff(-1)
        assert np.array_equal(ga.cpu().numpy(), Ah), ("deletion", e)
        assert np.array_equal(gb.cpu().numpy(), Bh), ("deletion", e)
        ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "hilo"])
def test_small_affected_area_uses_the_transpose_copy(prec):
    """Updates into sinks without out-edges have A_hat = {j}: only row j goes through the
    streaming update and the pairs (y, j) are copied from (j, y). S matches the oracle's
    Inc-uSR (K-matched) and the recompute, and stays exactly symmetric."""
    n, K = 500, 15
    s, d = W.chung_lu(n, 2500, seed=931)
    outdeg = np.bincount(s, minlength=n)
    indeg = np.bincount(d, minlength=n)
    sinks = [x for x in range(n) if outdeg[x] == 0 and indeg[x] >= 2][:3]
    assert len(sinks) == 3
    es = set(zip(s.tolist(), d.tolist()))
    ups = [(next(a for a in range(n) if a != j and (a, j) not in es), j, 1) for j in sinks[:2]]
    ups.append((next(a for (a, b) in sorted(es) if b == sinks[2]), sinks[2], -1))
    ctx = ctx_for(n, s, d, s_prec=prec, K=K)
    tr = EdgeTracker(n, s, d)
    S_or = O.fixed_point(tr.Q(), C)
    for (i, j, op) in ups:
        cs, cd = tr.arrays()
        Qd = Gr.transition_matrix(n, cs, cd, dense=True)
        S_or, _ = OI.inc_usr(Qd, S_or, np.bincount(cd, minlength=n), i, j, C, K, op=op)
        st = ctx.apply_edge_update(i, j, op, stats=True)
        tr.apply(i, j, op)
        assert st["aff_A"] == 1 and st["pairs"] == 2 * st["aff_B"] - 1
        S = ctx.S().cpu().numpy()
        assert np.array_equal(S, S.T)
        assert maxabs(S, S_or) < (1e-12 if prec == "fp64" else 1e-9)
        assert maxabs(S, tr.exact(C)) < TOL
    ctx.close()


def test_node_insertion_cases_unit():
    n = 300
    s, d = W.chung_lu(n, 1200, seed=51)
    ctx = ctx_for(n, s, d, s_prec="fp64", node_cap=n + 16)
    tr = EdgeTracker(n, s, d)
    seq = [(5, n, 1), (n + 1, 7, 1), (n + 2, n + 3, 1), (n, 9, 1), (2, n + 1, 1),
           (n + 4, n, 1), (3, 8, 1)]
    for i, j, o in seq:
        if (i, j) in tr.es:
            continue
        st = ctx.apply_edge_update(i, j, o, stats=True)
        tr.apply(i, j, o)
        assert ctx.sizes()[0] == tr.n
        assert maxabs(ctx.S().cpu().numpy(), tr.exact(C)) < TOL, (i, j, st)


def test_batches_match_oracle_plan_and_recompute():
    n = 300
    s, d = W.chung_lu(n, 1500, seed=61)
    batches, counts = W.batch_stream(n, s, d, 3, 150, 62)
    ctx = ctx_for(n, s, d, s_prec="fp64", node_cap=counts[-1] + 8, fused_batch=False)
    tr = EdgeTracker(n, s, d)
    for (bi, bj, bo), nn in zip(batches, counts):
        cs, cd = tr.arrays()
        plan_or, n_new = OI.plan_batch(tr.n, cs, cd, bi, bj, bo)
        st = ctx.apply_batch(bi, bj, bo, stats=True)
        plan = ctx.last_plan()
        assert [(b["case"], b["op"], b["j"], b["dj"], b["I"]) for b in plan] == \
               [(b["case"], b["op"], b["j"], b["dj"], b["I"]) for b in plan_or]
        plus, minus = OI.net_update(bi, bj, bo)
        for (i, j) in minus:
            tr.apply(i, j, -1)
        for (i, j) in plus:
            tr.apply(i, j, 1)
        tr.n = nn
        assert st["n_after"] == nn
        assert maxabs(ctx.S().cpu().numpy(), tr.exact(C)) < TOL


def _pad(v, n):
    return np.concatenate([v, np.zeros(n - len(v))])


def test_column_mode_all_cases():
    """Algorithm 7 in column mode for every case of a unit update: an insertion between
    existing nodes (C0), into a new sink (C1), from a new source (C2), between two new nodes
    (C3), and a deletion (Theorem 9). The Delta S columns (float64 single columns and the
    float32 list) match the oracle's column method at the same K and PartialSim depth, and
    with a deep PartialSim the converged recompute's change of S (1e-6); the new nodes' own
    columns included."""
    n, K = 1500, 10
    s, d = W.chung_lu(n, 9000, seed=991)
    es = set(zip(s.tolist(), d.tolist()))
    i0, j0 = next((a, b) for a in range(3, n) for b in range(7, n)
                  if a != b and (a, b) not in es)
    dele = sorted(es)[17]
    seq = [(i0, j0, 1), (5, n, 1), (n + 1, 9, 1), (n + 2, n + 3, 1), (dele[0], dele[1], -1)]
    lit = ctx_for(n, s, d, mode="column", K=K, K_ps=K, node_cap=n + 8)
    deep = ctx_for(n, s, d, mode="column", K=K, K_ps=40, node_cap=n + 8)
    cur_n = n
    cur_s, cur_d = s.astype(np.int64), d.astype(np.int64)
    for (i, j, op) in seq:
        st = lit.apply_edge_update(i, j, op, stats=True)
        deep.apply_edge_update(i, j, op)
        n2, s2, d2 = Gr.apply_edges(cur_n, cur_s, cur_d, [i], [j], [op])
        assert lit.sizes()[0] == n2 and st["n_after"] == n2
        cols = np.unique(np.concatenate([W.column_sample(cur_n, 24, seed=992 + i),
                                         [i, j, 0, n2 - 1]])).astype(np.int32)
        cols = cols[cols < n2]
        # oracle, K-matched: Algorithm 7 (insertions) or the block column method (deletion)
        if op > 0:
            ref = np.stack([OI.inc_sr_all_p_column(cur_n, cur_s, cur_d, np.zeros(cur_n), int(x),
                                                   [(i, j)], C, K) for x in cols], 1)
        else:
            ref = OI.delta_columns_batch(cur_n, cur_s, cur_d, [i], [j], [-1], cols, C, K, K)
        got64 = np.stack([lit.query_column(int(x), what="delta").cpu().numpy() for x in cols], 1)
        got32 = lit.query_columns(cols).double().cpu().numpy().T
        assert got64.shape == ref.shape == (n2, len(cols))
        assert maxabs(got64, ref) < 1e-12, (i, j, op)
        assert maxabs(got32, ref) < 1e-7, (i, j, op)
        # converged: the change of S* (new nodes' old columns are zero)
        Qo = Gr.transition_matrix(cur_n, cur_s, cur_d)
        Qn = Gr.transition_matrix(n2, s2, d2)
        exact = np.stack([O.single_source(Qn, int(x), C) -
                          (_pad(O.single_source(Qo, int(x), C), n2) if x < cur_n else 0.0)
                          for x in cols], 1)
        gd = np.stack([deep.query_column(int(x), what="delta").cpu().numpy() for x in cols], 1)
        assert maxabs(gd, exact) < TOL, (i, j, op, maxabs(gd, exact))
        cur_n, cur_s, cur_d = n2, s2.astype(np.int64), d2.astype(np.int64)
    lit.close()
    deep.close()


def long_block_batches(n, s, d):
    """Three batches whose similar-sink blocks have more than 60 sources each: 130 existing
    sources into an existing sink (C0), 70 existing sources into a new sink (C1), 65 new
    sources into an existing sink (C2), 64 new sources into a new sink (C3); then 70
    deletions from a sink that keeps 64 in-edges (d_j > delta) beside 61 insertions into
    another sink; then the deletion of all 64 in-edges of that sink (d_j = delta)."""
    es = set(zip(s.tolist(), d.tolist()))
    b1 = [(a, 0) for a in range(1, n) if (a, 0) not in es][:130]
    b1 += [(a, n) for a in range(10, 80)]
    b1 += [(n + 1 + t, 7) for t in range(65)]
    b1 += [(n + 67 + t, n + 66) for t in range(64)]
    es1 = es | set(b1)
    d2 = [(a, 0, -1) for (a, _) in b1[:70]]
    i2 = [(a, 7, 1) for a in range(100, n) if (a, 7) not in es1][:61]
    es2 = (es1 - {(a, 0) for a, _, _ in d2}) | {(a, 7) for a, _, _ in i2}
    d3 = sorted((a, 0, -1) for (a, j) in es2 if j == 0)
    out = [([a for a, _ in b1], [j for _, j in b1], [1] * len(b1))]
    for bt in (d2 + i2, d3):
        out.append(([e[0] for e in bt], [e[1] for e in bt], [e[2] for e in bt]))
    return out


@pytest.mark.parametrize("fused,chunk", [(False, 64), (True, 2), (True, 64)])
def test_long_blocks_are_single_updates(fused, chunk):
    """Blocks of more than 60 sources (device-resident source lists) in every case: the
    library's plan equals the oracle's unsplit Algorithm 6 plan, S matches the oracle's
    Inc-bSR at the same K (K-matched, 1e-12) and the converged recompute (1e-6)."""
    n, K = 400, 15
    s, d = W.chung_lu(n, 2400, seed=81)
    batches = long_block_batches(n, s, d)
    ctx = ctx_for(n, s, d, s_prec="fp64", K=K, node_cap=n + 140, fused_batch=fused,
                  batch_chunk=chunk)
    tr = EdgeTracker(n, s, d)
    S_or = O.fixed_point(tr.Q(), C)
    assert maxabs(ctx.S().cpu().numpy(), S_or) < 1e-13
    sizes = []
    for bi, bj, bo in batches:
        cs, cd = tr.arrays()
        S_or, plan_or = OI.inc_bsr(tr.n, cs, cd, S_or, bi, bj, bo, C, K)
        ctx.apply_batch(bi, bj, bo)
        plan = ctx.last_plan()
        assert [(b["case"], b["op"], b["j"], b["dj"], b["I"]) for b in plan] == \
               [(b["case"], b["op"], b["j"], b["dj"], b["I"]) for b in plan_or]
        sizes += [(b["case"], b["op"], len(b["I"])) for b in plan]
        plus, minus = OI.net_update(bi, bj, bo)
        for (i, j) in minus:
            tr.apply(i, j, -1)
        for (i, j) in plus:
            tr.apply(i, j, 1)
        S = ctx.S().cpu().numpy()
        assert maxabs(S, S_or) < 1e-12
        assert maxabs(S, tr.exact(C)) < TOL
    assert sizes == [(0, 1, 130), (2, 1, 65), (1, 1, 70), (3, 1, 64), (0, -1, 70), (0, 1, 61),
                     (0, -1, 64)]
    ctx.close()


def test_column_mode_delta_columns():
    n = 1500
    K = 10
    s, d = W.chung_lu(n, 9000, seed=71)
    ii, jj = W.insertion_stream(n, s, d, 3, seed=72)
    cols = W.column_sample(n, 40, seed=73, extra=[0, n - 1])
    deep = ctx_for(n, s, d, mode="column", K=K, K_ps=30)
    lit = ctx_for(n, s, d, mode="column", K=K, K_ps=K)
    cur_s, cur_d = s.astype(np.int64), d.astype(np.int64)
    for i, j in zip(ii.tolist(), jj.tolist()):
        c = np.unique(np.concatenate([cols, [i, j]])).astype(np.int32)
        deep.apply_edge_update(i, j, 1)
        lit.apply_edge_update(i, j, 1)
        got = deep.query_columns(c).double().cpu().numpy().T
        n2, s2, d2 = Gr.apply_edges(n, cur_s, cur_d, [i], [j], [1])
        Qo = Gr.transition_matrix(n, cur_s, cur_d)
        Qn = Gr.transition_matrix(n, s2, d2)
        exact = np.stack([O.single_source(Qn, x, C) - O.single_source(Qo, x, C) for x in c], 1)
        # float32 output columns: tolerance covers float32 rounding of the entries
        assert maxabs(got, exact) < TOL + 1e-7
        # the paper's literal Algorithm 7 (PartialSim depth K) against the oracle's own
        ref = OI.delta_columns_c0(n, cur_s, cur_d, i, j, c, C, K, K)
        got_lit = lit.query_columns(c).double().cpu().numpy().T
        assert maxabs(got_lit, ref) < 1e-6
        # float64 single column
        dc = deep.query_column(int(c[1]), what="delta").cpu().numpy()
        assert maxabs(dc, exact[:, 1]) < TOL
        cur_s, cur_d = s2.astype(np.int64), d2.astype(np.int64)


def _existing_batch(n, s, d, seed, n_ins, n_del, shared):
    """Insertions of non-edges (the first `shared` into one sink) and deletions of existing
    edges, all between existing nodes."""
    g = W.rng(seed)
    es = set(zip(s.tolist(), d.tolist()))
    bi, bj, bo = [], [], []
    sink = int(g.integers(n))
    while len(bi) < n_ins:
        a = int(g.integers(n))
        b = sink if len(bi) < shared else int(g.integers(n))
        if a != b and (a, b) not in es and (a, b) not in set(zip(bi, bj)):
            bi.append(a)
            bj.append(b)
            bo.append(1)
    for e in g.choice(len(s), size=n_del, replace=False).tolist():
        bi.append(int(s[e]))
        bj.append(int(d[e]))
        bo.append(-1)
    return bi, bj, bo


@pytest.mark.parametrize("chunk", [1, 5, 64, 0])
def test_column_batch_matches_oracle(chunk):
    """Column mode, a batch between existing nodes: Algorithm 6's blocks with the column
    method inside, summed over the blocks on FP64 matrix cores, against the oracle's same
    computation (same K and PartialSim depth) on a ragged shape (n = 1500 nodes, 70 columns);
    chunk 1 runs one pass per block, chunk 64 one pass for the batch, 0 the column-mode
    default, ceil(512 / 2(K+1)) = 24 blocks per pass at K = 10."""
    n, K, Kps = 1500, 10, 30
    s, d = W.chung_lu(n, 9000, seed=91)
    bi, bj, bo = _existing_batch(n, s, d, seed=92, n_ins=14, n_del=6, shared=4)
    cols = W.column_sample(n, 66, seed=93, extra=[bj[0], bi[0], 0, n - 1])[:70]
    ctx = ctx_for(n, s, d, mode="column", K=K, K_ps=Kps, batch_chunk=chunk)
    if chunk == 0:
        chunk = ctx.config().batch_chunk
        assert chunk == 24
    out, st = ctx.apply_batch_columns(bi, bj, bo, cols, stats=True)
    got = out.cpu().numpy().T
    ref = OI.delta_columns_batch(n, s.astype(np.int64), d.astype(np.int64), bi, bj, bo, cols, C,
                                 K, Kps)
    scale = np.abs(ref).max()
    assert scale > 0 and maxabs(got, ref) < 1e-12 * scale + 1e-15
    assert st["fused_passes"] == -(-st["lowrank_blocks"] // chunk)
    assert ctx.sizes() == (n, len(s) + 14 - 6)
    ctx.close()


def test_column_batch_rejections_leave_state():
    n = 300
    s, d = W.chung_lu(n, 1200, seed=94)
    ctx = ctx_for(n, s, d, mode="column", K=5, K_ps=10, node_cap=n + 8)
    from paper_1711_00121_amd._lib import SR_EMODE, SR_ERANGE, SimRankError
    with pytest.raises(SimRankError) as e:
        ctx.apply_batch_columns([1, 2], [n, 3], [1, 1], [0, 1])   # creates node n
    assert e.value.status == SR_EMODE
    with pytest.raises(SimRankError) as e:
        ctx.apply_batch_columns([1], [2] if (1, 2) not in set(zip(s.tolist(), d.tolist()))
                                else [3], [1], [0, n])
    assert e.value.status == SR_ERANGE
    assert ctx.sizes() == (n, len(s))
    dense = ctx_for(n, s, d, s_prec="fp64")
    with pytest.raises(SimRankError) as e:
        dense.apply_batch_columns([1], [2], [1], [0])
    assert e.value.status == SR_EMODE
    ctx.close()
    dense.close()


def test_column_batch_degenerate_inputs():
    """An empty batch gives zero columns and leaves the graph; an empty column list still
    applies the batch (the next batch's columns then follow the updated graph)."""
    n = 400
    s, d = W.chung_lu(n, 1600, seed=97)
    ctx = ctx_for(n, s, d, mode="column", K=5, K_ps=10)
    out = ctx.apply_batch_columns([], [], [], [0, 5, n - 1])
    assert out.shape == (3, n) and float(out.abs().max()) == 0.0
    assert ctx.sizes() == (n, len(s))
    bi, bj, bo = _existing_batch(n, s, d, 98, 4, 2, 2)
    ctx.apply_batch_columns(bi, bj, bo, [])
    assert ctx.sizes() == (n, len(s) + 2)
    # a second batch on the updated graph, against the oracle started from it
    s2 = np.asarray([a for a, b in zip(s.tolist(), d.tolist())
                     if (a, b) not in set(zip(bi[4:], bj[4:]))] + bi[:4], dtype=np.int64)
    d2 = np.asarray([b for a, b in zip(s.tolist(), d.tolist())
                     if (a, b) not in set(zip(bi[4:], bj[4:]))] + bj[:4], dtype=np.int64)
    ci, cj, co = _existing_batch(n, s2, d2, 99, 3, 1, 2)
    cols = np.array([0, 7, 200, n - 1])
    got = ctx.apply_batch_columns(ci, cj, co, cols).cpu().numpy().T
    ref = OI.delta_columns_batch(n, s2, d2, ci, cj, co, cols, C, 5, 10)
    assert maxabs(got, ref) < 1e-12 * max(1.0, float(np.abs(ref).max()))
    ctx.close()


@pytest.mark.parametrize("K,n", [(0, 700), (3, 701), (4, 700), (6, 702), (8, 700), (10, 703),
                                 (12, 700), (15, 701)])
def test_column_kernel_every_depth(K, n):
    """Delta S columns at every series depth the column kernel specialises on (ceil(2 (K + 1)
    / 4) = 1 .. 8 k-steps), on ragged shapes: n = 700 .. 703 nodes (the last 64-node strip is
    partial; rows of n floats are 16-byte aligned only for n = 700, the other sizes take the
    4-byte stores) and 70 columns (the last row tile is partial)."""
    s, d = W.chung_lu(n, 4200, seed=81)
    ii, jj = W.insertion_stream(n, s, d, 1, seed=82)
    i, j = int(ii[0]), int(jj[0])
    c = W.column_sample(n, 68, seed=83, extra=[i, j])
    ctx = ctx_for(n, s, d, mode="column", K=K, K_ps=12)
    ctx.apply_edge_update(i, j, 1)
    got = ctx.query_columns(c).double().cpu().numpy().T
    ref = OI.delta_columns_c0(n, s.astype(np.int64), d.astype(np.int64), i, j, c, C, K, 12)
    # same K and K_ps on both sides in float64; the output is rounded to float32
    assert np.all(np.abs(got - ref) <= 2.0 ** -24 * np.abs(ref) * 1.01 + 1e-13)
    ctx.close()


def test_backward_matches_oracle_gradient():
    n = 200
    s, d = W.chung_lu(n, 1000, seed=81)
    w = W.lognormal_weights(len(s), seed=82)
    a, b, t = W.loss_pairs(n, 120, seed=83)
    from paper_1711_00121_amd import Context, simrank_pairs
    ctx = Context(n, s, d, weight=w, s_prec="fp64")
    g_or, S_or, _ = OA.grad_weights_dense(n, s, d, w, a, b, t, C)
    assert maxabs(ctx.S().cpu().numpy(), S_or) < 1e-13
    wt = torch.tensor(w, dtype=torch.float64, device="cuda", requires_grad=True)
    vals = simrank_pairs(wt, ctx, a, b)
    loss = ((vals - torch.tensor(t, device="cuda")) ** 2).sum()
    loss.backward()
    g = wt.grad.cpu().numpy()
    assert maxabs(g, g_or) < 1e-10 * max(1.0, np.abs(g_or).max())
    # Euler identity per sink
    for x in range(n):
        sel = d == x
        if sel.any():
            assert abs(np.sum(w[sel] * g[sel])) < 1e-12


def test_errors_leave_state_unchanged():
    from paper_1711_00121_amd._lib import SimRankError
    n = 100
    s, d = W.chung_lu(n, 400, seed=91)
    ctx = ctx_for(n, s, d, s_prec="fp64")
    S0 = ctx.S().cpu().numpy()
    e0 = (int(s[0]), int(d[0]))
    for args, code in [((e0[0], e0[1], 1), -3), ((0, 0, 1), -5), ((0, n + 5, 1), -2),
                       ((1, 2, 3), -1)]:
        if args == (1, 2, 1):
            continue
        with pytest.raises(SimRankError) as ei:
            ctx.apply_edge_update(*args)
        assert ei.value.status == code
    es = set(zip(s.tolist(), d.tolist()))
    missing = next((a, b) for a in range(n) for b in range(n) if a != b and (a, b) not in es)
    with pytest.raises(SimRankError) as ei:
        ctx.apply_edge_update(missing[0], missing[1], -1)
    assert ei.value.status == -4
    with pytest.raises(SimRankError):
        ctx.apply_batch([1, 1], [2, 2], [1, 1])
    assert np.array_equal(ctx.S().cpu().numpy(), S0)


def test_fused_batch_slot_cap_flushes_early():
    """A chunk holds at most 2 chunk + 32 blocks that read columns of S; one more forces an
    early fused pass. One C0 insertion (deferred) followed by 40 insertions into 40 new sinks
    (C1 blocks, which read the deferred block's corrections) with batch_chunk = 3 (cap 38):
    the 38th reading block flushes the chunk with its one deferred block (the batch's only
    fused pass), and the last C1 blocks start a new chunk whose corrections are zero. S must
    match the oracle's Inc-bSR at the same K."""
    n = 300
    K = 15
    s, d = W.chung_lu(n, 1500, seed=65)
    es = set(zip(s.tolist(), d.tolist()))
    g = W.rng(66)
    while True:
        i, j = (int(v) for v in g.integers(n, size=2))
        if i != j and (i, j) not in es:
            break
    srcs = g.choice(n, size=40, replace=True)
    bi = [i] + [int(x) for x in srcs]
    bj = [j] + list(range(n, n + 40))
    bo = [1] * len(bi)
    ctx = ctx_for(n, s, d, s_prec="fp64", node_cap=n + 40, fused_batch=True, batch_chunk=3,
                  K=K)
    st = ctx.apply_batch(bi, bj, bo, stats=True)
    assert st["blocks_case"][0] == 1 and st["blocks_case"][1] == 40
    assert st["fused_passes"] == 1 and st["lowrank_blocks"] == 1
    S_or, _ = OI.inc_bsr(n, s.astype(np.int64), d.astype(np.int64),
                         O.fixed_point(Gr.transition_matrix(n, s, d), C), bi, bj, bo, C, K)
    assert maxabs(ctx.S().cpu().numpy(), S_or) < 1e-12
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "hilo"])
@pytest.mark.parametrize("chunk", [1, 3, 64])
def test_fused_batches_match_oracle(prec, chunk):
    """Fused form of Algorithm 6: low-rank blocks deferred into stacked panels, S columns
    corrected by the deferred terms before each gamma, one S pass per chunk.

    This stream's K = 15 truncation error (2.5e-6, the oracle's own Inc-bSR at K = 15 shows
    the same) exceeds 1e-6, so parity is checked twice: at K = 15 against the oracle's
    K-truncated Inc-bSR (same method, tight tolerance), and at K = 40 against the converged
    recompute at 1e-6. Chunk 1 makes every pass a single block."""
    n = 300
    s, d = W.chung_lu(n, 1500, seed=63)
    batches, counts = W.batch_stream(n, s, d, 3, 150, 64)
    ctx15 = ctx_for(n, s, d, s_prec=prec, node_cap=counts[-1] + 8, fused_batch=True,
                    batch_chunk=chunk, K=15)
    ctx40 = ctx_for(n, s, d, s_prec=prec, node_cap=counts[-1] + 8, fused_batch=True,
                    batch_chunk=chunk, K=40)
    tr = EdgeTracker(n, s, d)
    S_or = O.fixed_point(Gr.transition_matrix(n, s, d), C)
    for (bi, bj, bo), nn in zip(batches, counts):
        cs, cd = tr.arrays()
        S_or, _ = OI.inc_bsr(tr.n, cs, cd, S_or, bi, bj, bo, C, 15)
        st = ctx15.apply_batch(bi, bj, bo, stats=True)
        ctx40.apply_batch(bi, bj, bo)
        plus, minus = OI.net_update(bi, bj, bo)
        for (i, j) in minus:
            tr.apply(i, j, -1)
        for (i, j) in plus:
            tr.apply(i, j, 1)
        tr.n = nn
        assert st["fused_passes"] == -(-st["lowrank_blocks"] // chunk)
        # a pass covers the nodes with a nonzero panel row in one of its blocks: at most all
        assert 0 < st["pass_entries"] <= st["lowrank_blocks"] * nn * (nn + 1) // 2
        S15 = ctx15.S().cpu().numpy()
        # every fused pass, one block or many, writes (a, b) and (b, a) from one sum
        assert np.array_equal(S15, S15.T)
        assert maxabs(S15, S_or) < (1e-12 if prec == "fp64" else 1e-9)
        assert maxabs(ctx40.S().cpu().numpy(), tr.exact(C)) < TOL


@pytest.mark.parametrize("update_prec", ["fp64", "fp32"])
def test_fused_passes_cover_the_reached_nodes_only(update_prec):
    """Nodes without in-edges never enter a block's series (their S rows stay (1 - C) e_a), so
    a fused pass skips them: with half the nodes given no in-edges, the passes cover fewer
    entries than the whole square, and S still matches the oracle's Inc-bSR and stays exactly
    symmetric; the rows of the skipped nodes are unchanged."""
    n = 400
    s, d = W.chung_lu(n, 2400, seed=71)
    keep = d < n // 2  # nodes n/2 .. n-1 keep only their out-edges
    s, d = s[keep], d[keep]
    tr = EdgeTracker(n, s, d)
    bi, bj, bo = (np.asarray(x) for x in _existing_batch(n, s, d, seed=72, n_ins=60, n_del=20,
                                                          shared=10))
    ok = bj < n // 2  # insert and delete only into the first half
    bi, bj, bo = bi[ok], bj[ok], bo[ok]
    ctx = ctx_for(n, s, d, s_prec="fp64", fused_batch=True, batch_chunk=4, K=15,
                  update_prec=update_prec)
    S0 = ctx.S().cpu().numpy()
    st = ctx.apply_batch(bi, bj, bo, stats=True)
    S = ctx.S().cpu().numpy()
    S_or, _ = OI.inc_bsr(n, s.astype(np.int64), d.astype(np.int64),
                         O.fixed_point(Gr.transition_matrix(n, s, d), C), bi, bj, bo, C, 15)
    full = st["lowrank_blocks"] * n * (n + 1) // 2
    print(f"pass entries {st['pass_entries']} of {full}", flush=True)
    assert st["pass_entries"] < full * 0.6
    # float32 matrix cores: products of the rounded panel, summed in float32 per pass
    assert maxabs(S, S_or) < (1e-12 if update_prec == "fp64" else 1e-6)
    assert np.array_equal(S, S.T)
    sinkless = np.setdiff1d(np.arange(n // 2, n), np.asarray(tr.arrays()[1]))
    assert np.array_equal(S[sinkless], S0[sinkless])
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "hilo"])
@pytest.mark.parametrize("K", [15, 10])
def test_tile_skip_is_bit_exact(prec, K):
    """xi_k vanishes outside the nodes k out-steps from a block's sink, so a fused pass skips,
    per 128 x 128 tile, the k-steps whose xi factors are zero on both of the tile's row ranges.
    The skipped products are exact zeros: two contexts, tile skipping on and off, take the same
    two batches at n = 3000 (the reached nodes span ~17 tiles and a ragged tail; chunks of 8
    blocks) and hold the same S bit for bit, after each batch. At K = 10 the panel's last
    columns are zero padding (22 of 32), skipped too, and not counted as skipped work."""
    n = 3000
    s, d = W.chung_lu(n, 24000, seed=81)
    kw = dict(s_prec=prec, fused_batch=True, batch_chunk=8, K=K, edge_cap=24000 + 2000)
    on = ctx_for(n, s, d, **kw)
    off = ctx_for(n, s, d, tile_skip=False, **kw)
    tr = EdgeTracker(n, s, d)
    steps = (K + 2) // 2
    for b in range(2):
        cs, cd = tr.arrays()
        bi, bj, bo = (np.asarray(x) for x in _existing_batch(n, cs, cd, seed=82 + b, n_ins=150,
                                                              n_del=50, shared=20))
        sa = on.apply_batch(bi, bj, bo, stats=True)
        sb = off.apply_batch(bi, bj, bo, stats=True)
        plus, minus = OI.net_update(bi, bj, bo)
        for (i, j) in minus:
            tr.apply(i, j, -1)
        for (i, j) in plus:
            tr.apply(i, j, 1)
        frac = sa["pass_skipped"] / max(sa["pass_entries"] * steps, 1)
        print(f"K={K} {prec} batch {b}: {sa['fused_passes']} passes, skipped {frac:.3f} of "
              f"the entry k-steps", flush=True)
        assert sa["pass_entries"] == sb["pass_entries"] and sa["pairs"] == sb["pairs"]
        assert sb["pass_skipped"] == 0 and 0 < sa["pass_skipped"] < sa["pass_entries"] * steps
        Sa, Sb = on.S().cpu().numpy(), off.S().cpu().numpy()
        assert np.array_equal(Sa.view(np.uint64), Sb.view(np.uint64))
        assert np.array_equal(Sa, Sa.T)
    on.close()
    off.close()
