"""The fused batch's launch machinery through the C ABI: K-step series chains replayed from
captured HIP graphs give bit-for-bit the S of plain launches (many replays, with the batch's
other launches and synchronisations between them) and match the oracle's Inc-bSR; every GEMM
tile variant gives the same S; the autotuner leaves S unchanged, caches its choice, and a
tuned context still matches the oracle."""
import numpy as np
import pytest

import workloads as W
from oracle import graph as Gr
from oracle import incremental as OI
from oracle import simrank as O

from _util import EdgeTracker, maxabs

pytestmark = pytest.mark.gpu

C = 0.6


def ctx_for(n, s, d, **kw):
    from paper_1711_00121_amd import Context
    return Context(n, s, d, **kw)


def stream(n, m, seed, count=3, size=220):
    s, d = W.chung_lu(n, m, seed=seed)
    batches, counts = W.batch_stream(n, s, d, count, size, seed + 1, min_batch=size // 2)
    return s, d, batches, counts


def test_graph_replays_match_plain_launches_and_oracle():
    n, K = 400, 15
    s, d, batches, counts = stream(n, 2400, 1201)
    kw = dict(C=C, K=K, s_prec="fp64", node_cap=counts[-1] + 4, fused_batch=True, batch_chunk=6)
    g = ctx_for(n, s, d, graphs=True, **kw)
    p = ctx_for(n, s, d, graphs=False, **kw)
    tr = EdgeTracker(n, s, d)
    S_or = O.fixed_point(Gr.transition_matrix(n, s, d), C)
    total = 0
    for (bi, bj, bo), nn in zip(batches, counts):
        cs, cd = tr.arrays()
        S_or, _ = OI.inc_bsr(tr.n, cs, cd, S_or, bi, bj, bo, C, K)
        sg = g.apply_batch(bi, bj, bo, stats=True)
        sp = p.apply_batch(bi, bj, bo, stats=True)
        assert sg["series_replays"] == sg["lowrank_blocks"] and sp["series_replays"] == 0
        total += sg["series_replays"]
        plus, minus = OI.net_update(bi, bj, bo)
        for (i, j) in minus:
            tr.apply(i, j, -1)
        for (i, j) in plus:
            tr.apply(i, j, 1)
        tr.n = nn
        Sg = g.S().cpu().numpy()
        assert np.array_equal(Sg, p.S().cpu().numpy())
        assert maxabs(Sg, S_or) < 1e-12
    assert total > 100
    g.close()
    p.close()


def test_gemm_variants_give_the_same_S():
    """The tile variants differ in LDS chunk width and pitch, not in the order of the matrix
    core's sums, so S is the same bit for bit; and it matches the oracle."""
    n, K = 400, 15
    s, d, batches, counts = stream(n, 2400, 1203, count=2)
    results = []
    for variant in range(4):
        ctx = ctx_for(n, s, d, C=C, K=K, s_prec="hilo", node_cap=counts[-1] + 4, batch_chunk=7)
        ctx.set_tuning(5 + variant, variant)  # a different chunk each time, too
        for bi, bj, bo in batches:
            ctx.apply_batch(bi, bj, bo)
        results.append(ctx.S().cpu().numpy())
        ctx.close()
    tr = EdgeTracker(n, s, d)
    S_or = O.fixed_point(Gr.transition_matrix(n, s, d), C)
    for (bi, bj, bo), nn in zip(batches, counts):
        cs, cd = tr.arrays()
        S_or, _ = OI.inc_bsr(tr.n, cs, cd, S_or, bi, bj, bo, C, K)
        plus, minus = OI.net_update(bi, bj, bo)
        for (i, j) in minus:
            tr.apply(i, j, -1)
        for (i, j) in plus:
            tr.apply(i, j, 1)
        tr.n = nn
    for r in results:
        assert maxabs(r, S_or) < 1e-9
    # the chunk changes the deferral (and so the order of additions) but not the variant
    ctx_a = ctx_for(n, s, d, C=C, K=K, s_prec="fp64", node_cap=counts[-1] + 4)
    ctx_b = ctx_for(n, s, d, C=C, K=K, s_prec="fp64", node_cap=counts[-1] + 4)
    ctx_a.set_tuning(9, 0)
    ctx_b.set_tuning(9, 3)
    for bi, bj, bo in batches:
        ctx_a.apply_batch(bi, bj, bo)
        ctx_b.apply_batch(bi, bj, bo)
    assert np.array_equal(ctx_a.S().cpu().numpy(), ctx_b.S().cpu().numpy())


def test_autotuner_keeps_S_and_caches(tmp_path):
    from paper_1711_00121_amd import _lib as L
    n, K = 1500, 15
    s, d, batches, counts = stream(n, 9000, 1205, count=1, size=300)
    ctx = ctx_for(n, s, d, C=C, K=K, s_prec="hilo", node_cap=counts[-1] + 4)
    S0 = ctx.S().cpu().numpy()
    path = str(tmp_path / "tuning.json")
    info = ctx.tune(chunks=(4, 8, 16), path=path)
    assert not info["cached"] and len(info["table"]) == 12
    assert info["batch_chunk"] in (4, 8, 16) and info["variant"] in (0, 1, 2, 3)
    assert all(t["gemm_ms"] > 0 for t in info["table"])
    assert np.array_equal(ctx.S().cpu().numpy(), S0)
    again = ctx.tune(chunks=(4, 8, 16), path=path)
    assert again["cached"] and again["batch_chunk"] == info["batch_chunk"]
    with pytest.raises(L.SimRankError):
        ctx.time_fused(7, 4)
    with pytest.raises(L.SimRankError):
        ctx.set_tuning(0, 0)
    tr = EdgeTracker(n, s, d)
    bi, bj, bo = batches[0]
    ctx.apply_batch(bi, bj, bo)
    plus, minus = OI.net_update(bi, bj, bo)
    for (i, j) in minus:
        tr.apply(i, j, -1)
    for (i, j) in plus:
        tr.apply(i, j, 1)
    tr.n = counts[0]
    assert maxabs(ctx.S().cpu().numpy(), tr.exact(C)) < 1e-6
    ctx.close()


def test_mfma_f32_lane_layout():
    """v_mfma_f32_16x16x4f32: lane l supplies A[l%16][l//16] and B[l//16][l%16]; slot v of lane
    l holds D[4*(l//16) + v][l%16]. The float32 fused pass relies on this layout."""
    import ctypes as Cc
    import torch
    from paper_1711_00121_amd import _lib as L
    a = torch.arange(64, dtype=torch.float32, device="cuda") * 0.5 + 1.0
    b = torch.arange(64, dtype=torch.float32, device="cuda") * 0.25 - 3.0
    out = torch.empty(256, dtype=torch.float32, device="cuda")
    assert L.load().sr_mfma_layout_probe_f32(Cc.c_void_p(a.data_ptr()), Cc.c_void_p(b.data_ptr()),
                                             Cc.c_void_p(out.data_ptr()), None) == 0
    torch.cuda.synchronize()
    A = np.zeros((16, 4))
    B = np.zeros((4, 16))
    for l in range(64):
        A[l % 16, l // 16] = a[l].item()
        B[l // 16, l % 16] = b[l].item()
    D = A @ B
    got = out.cpu().numpy()
    for l in range(64):
        for v in range(4):
            assert got[4 * l + v] == D[4 * (l // 16) + v, l % 16]


@pytest.mark.parametrize("prec", ["fp64", "hilo"])
def test_float32_update_passes(prec):
    """Fused passes on the float32 matrix cores: within 1e-6 of the oracle's Inc-bSR at the
    same K and of the converged recompute (K = 40), exactly symmetric; the gap to the float64
    passes is reported."""
    n = 400
    s, d, batches, counts = stream(n, 2400, 1207)
    kw = dict(C=C, s_prec=prec, node_cap=counts[-1] + 4, batch_chunk=6)
    f32 = ctx_for(n, s, d, K=15, update_prec="fp32", **kw)
    f64 = ctx_for(n, s, d, K=15, **kw)
    deep = ctx_for(n, s, d, K=40, update_prec="fp32", **kw)
    tr = EdgeTracker(n, s, d)
    S_or = O.fixed_point(Gr.transition_matrix(n, s, d), C)
    gap = 0.0
    for (bi, bj, bo), nn in zip(batches, counts):
        cs, cd = tr.arrays()
        S_or, _ = OI.inc_bsr(tr.n, cs, cd, S_or, bi, bj, bo, C, 15)
        for c in (f32, f64, deep):
            c.apply_batch(bi, bj, bo)
        plus, minus = OI.net_update(bi, bj, bo)
        for (i, j) in minus:
            tr.apply(i, j, -1)
        for (i, j) in plus:
            tr.apply(i, j, 1)
        tr.n = nn
        S = f32.S().cpu().numpy()
        assert np.array_equal(S, S.T)
        assert maxabs(S, S_or) < 1e-6
        gap = max(gap, maxabs(S, f64.S().cpu().numpy()))
        assert maxabs(deep.S().cpu().numpy(), tr.exact(C)) < 1e-6
    print(f"float32 passes ({prec} store): max gap to float64 passes {gap:.2e}")
    assert gap < 1e-6
