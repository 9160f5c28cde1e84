#!/usr/bin/env python3
"""Benchmark of incremental all-pairs SimRank on one MI355X.

Workload (default): directed Chung-Lu graph n = 50,000, m = 1,000,000 (exponent 2.1),
C = 0.6, K = 15, S stored as float32 value + float32 compensation (updates in float64);
one step = one batch of edge updates (sizes uniform in 1..4096; 40% new source, 20% new
sink, 10% both new, 30% between existing nodes; 25% of edges share a sink), applied by the
batch algorithm with deferred low-rank blocks and one fused pass over S per chunk.

Prints one JSON line: value = Delta S pair-updates/s (S entries updated per low-rank block,
summed, over wall time), plus edge updates/s, the plain per-edge GPU path on the same GPU and
accuracy, the roofline of the dominant kernel (live HIP events) and the oracle timed on the
host CPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("ΔS pair-updates/s + edge updates/s at n=50k vs plain GPU path; % HBM peak")
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=50_000)
    ap.add_argument("--m", type=int, default=1_000_000)
    ap.add_argument("--max-batch", type=int, default=4096)
    ap.add_argument("--chunk", type=int, default=64)
    ap.add_argument("--no-fused", action="store_true")
    ap.add_argument("--plain-edges", type=int, default=24)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this benchmark runs on one GPU only; --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return

    import numpy as np
    import torch

    import workloads as W
    from paper_1711_00121_amd import Context

    cfg = W.WORKLOADS[3]
    n, m, C, K = args.n, args.m, cfg["C"], cfg["K"]
    nb = args.warmup + args.steps + 1
    log(f"bench: generating Chung-Lu n={n} m={m} and {nb} batches")
    s, d = W.chung_lu(n, m, seed=1003)
    batches, counts = W.batch_stream(n, s, d, nb, args.max_batch, seed=2003)
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    ctx = Context(n, s, d, C=C, K=K, s_prec="hilo", node_cap=counts[-1] + 64,
                  edge_cap=m + sum(len(b[0]) for b in batches) + 1024,
                  fused_batch=not args.no_fused, batch_chunk=args.chunk)
    torch.cuda.synchronize()
    log(f"bench: init (S by fixed point on device) {time.perf_counter() - t0:.1f}s")

    for w in range(args.warmup):
        bi, bj, bo = batches[w]
        ctx.apply_batch(bi, bj, bo)
        torch.cuda.synchronize()
        log(f"bench: warmup batch {w} ({len(bi)} edges) done")

    ctx.profile(True)
    ctx.profile_read(reset=True)
    edges = 0
    pairs = 0
    lowrank = 0
    passes = 0
    n_nodes = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        bi, bj, bo = batches[args.warmup + k]
        st = ctx.apply_batch(bi, bj, bo, stats=True)
        edges += len(bi)
        pairs += st["pairs"]
        lowrank += st["lowrank_blocks"]
        passes += st["fused_passes"]
        n_nodes.append(st["n_after"])
        log(f"bench: step {k}: {len(bi)} edges, {st['blocks']} blocks "
            f"({st['lowrank_blocks']} low-rank), {st['fused_passes']} fused passes")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kern_ms, launches = ctx.profile_read(reset=True)
    ctx.profile(False)

    # Plain GPU path: the next batch's edges between existing nodes, one apply_edge_update each
    # (pruned single-edge update, same precision).
    bi, bj, bo = batches[args.warmup + args.steps]
    cur_n = ctx.sizes()[0]
    plain = [(int(a), int(b), int(o)) for a, b, o in zip(bi, bj, bo) if a < cur_n and b < cur_n]
    seen = set()
    sample = []
    for a, b, o in plain:
        if (a, b) in seen:
            continue
        seen.add((a, b))
        sample.append((a, b, o))
    # keep only edges whose net effect in the batch is this single op
    from collections import Counter
    cnt = Counter((int(a), int(b)) for a, b in zip(bi, bj))
    sample = [e for e in sample if cnt[(e[0], e[1])] == 1][:args.plain_edges]
    ctx.profile(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plain_pairs = 0
    for a, b, o in sample:
        st = ctx.apply_edge_update(a, b, o, stats=True)
        plain_pairs += st["pairs"]
    torch.cuda.synchronize()
    dt_plain = time.perf_counter() - t1
    plain_ms, plain_launches = ctx.profile_read(reset=True)
    ctx.profile(False)

    value = pairs / dt
    edge_rate = edges / dt
    plain_edge_rate = len(sample) / dt_plain if sample else None
    plain_pair_rate = plain_pairs / dt_plain if sample else None
    nf = float(np.mean(n_nodes))
    pld = 2 * (K + 1)
    if passes:
        # fused pass: Delta S is symmetric, so the method's work per low-rank block is its
        # n (n + 1) / 2 distinct entries at 2 (K + 1) multiply-adds each
        flops = nf * (nf + 1.0) * pld * lowrank
        achieved = flops / (kern_ms / 1e3) / 1e12
        roof = {"bound": "mfma", "achieved": round(achieved, 2), "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
                "traffic": traffic("lowrank_gemm_kernel"),
                "kernel": "lowrank_gemm_kernel (fused batch pass)",
                "launches": launches, "avg_ms": round(kern_ms / max(launches, 1), 3),
                "algorithmic": "n (n + 1) / 2 distinct entries x 4 (K + 1) flop per low-rank block"}
    else:
        achieved = 16.0 * pairs / (kern_ms / 1e3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic("lowrank_strip_kernel"),
                "kernel": "lowrank_strip_kernel", "launches": launches,
                "avg_ms": round(kern_ms / max(launches, 1), 3),
                "algorithmic": "16 B per pair-update (S value + compensation, read + write)"}
    plain_roof = None
    if sample:
        gbs = 16.0 * plain_pairs / (plain_ms / 1e3) / 1e9
        plain_roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                      "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                      "kernel": "lowrank_strip_kernel", "avg_ms": round(
                          plain_ms / max(plain_launches, 1), 3)}

    cpu = None
    if not args.no_cpu_baseline:
        applied = list(zip(batches[:args.warmup + args.steps],
                           counts[:args.warmup + args.steps]))
        cpu = cpu_baseline(n, s, d, applied, args.cpu_seconds)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "pair-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "n": n, "m": m, "C": C, "K": K,
                   "s_store": "f32 value + f32 compensation", "max_batch": args.max_batch,
                   "batch_chunk": args.chunk, "fused": not args.no_fused,
                   "parallelism": "single GPU"},
        "edge_updates_per_s": edge_rate,
        "edges": edges,
        "lowrank_blocks": lowrank,
        "fused_passes": passes,
        "plain_gpu": {"edges": len(sample), "edge_updates_per_s": plain_edge_rate,
                      "pair_updates_per_s": plain_pair_rate, "roofline": plain_roof},
        "speedup_edges_vs_plain": (edge_rate / plain_edge_rate) if plain_edge_rate else None,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def copy_calibration():
    """A plain device copy of 1 GiB, three times: the HBM counters of this launch calibrate
    FETCH_SIZE and WRITE_SIZE (bytes moved are known exactly)."""
    import torch
    x = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.neg(x, out=y)
    torch.cuda.synchronize()
    log(f"copy calibration: 3 x torch.neg over {x.numel() * 8} bytes read + written")


def traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, or None when the
    kernel's source has changed since the counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", f"{kernel}_pmc.md")
    src = os.path.join(ROOT, "paper_1711_00121_amd", "csrc", "update.hip")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_sha = re.search(r"source_sha256:\s*([0-9a-f]{64})", text)
    m_b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not (m_sha and m_b):
        return None
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != m_sha.group(1):
        return None
    return float(m_b.group(1))


def cpu_baseline(n, s, d, applied, seconds):
    """The oracle on the host: converged single-source columns S[:, x] of the graph after the
    timed batches (eq (17) by PartialSim to a tail C^(K+1) <= 1e-13), i.e. pair values of the
    updated S computed from scratch, timed on a bounded sample of columns."""
    import numpy as np

    from oracle import graph as Gr
    from oracle import incremental as OI
    from oracle import simrank as O

    cur_n, cur_s, cur_d = n, s, d
    for (bi, bj, bo), nn in applied:
        plus, minus = OI.net_update(bi, bj, bo)
        cur_n, cur_s, cur_d = Gr.apply_edges(
            cur_n, cur_s, cur_d, [e[0] for e in plus + minus], [e[1] for e in plus + minus],
            [1] * len(plus) + [-1] * len(minus), n_new=nn)
    Q = Gr.transition_matrix(cur_n, cur_s, cur_d)
    rng = np.random.default_rng(7)
    t0 = time.perf_counter()
    cols = 0
    while time.perf_counter() - t0 < seconds:
        O.single_source(Q, int(rng.integers(cur_n)), 0.6, tol=1e-13)
        cols += 1
    dt = time.perf_counter() - t0
    return {"value": cols * cur_n / dt, "unit": "pair-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{cols} converged single-source columns S[:, x] (x uniform) of the "
                      f"graph after the timed batches (n={cur_n}), oracle PartialSim to a "
                      f"tail <= 1e-13, {dt:.1f} s on one host thread (scipy sparse products "
                      f"are single-threaded)"}


if __name__ == "__main__":
    main()
