#!/usr/bin/env python3
"""Benchmark of incremental all-pairs SimRank on one MI355X.

Default workload (--workload batch): directed Chung-Lu graph n = 50,000, m = 1,000,000
(exponent 2.1), C = 0.6, K = 15, S stored as float32 value + float32 compensation (updates
in float64); one step = one batch of edge updates (sizes uniform in 1..4096; 40% new
source, 20% new sink, 10% both new, 30% between existing nodes; 25% of edges share a sink),
applied by the batch algorithm with deferred low-rank blocks and fused passes over S.

Prints one JSON line: value = Delta S pair-updates/s (S entries updated per low-rank block,
summed, over wall time), plus edge updates/s, the plain per-edge GPU path on the same GPU and
accuracy, the roofline of the dominant kernel (HIP events on the library's stream) and the
oracle timed on the host CPU.

The other workloads of the method are measured the same way with --workload:
  stream   n = 20k, m = 200k, 1,000 single-edge updates (70% insert), pruned, K = 15
  columns  n = 1M, m = 10M, column-by-column mode (no stored S), K = 10, PartialSim depth
           30; per insertion 65,536 Delta S columns in blocks of 8,192, float32 output
  columns_batch  the columns graph; per step one batch between existing nodes (48
           insertions, 16 of them into one sink, and 16 deletions) applied block by block,
           returning the batch's float64 Delta S columns for 8,192 columns
  forest   the stream's graph (n = 20k, m = 200k); one step computes all-pairs S by seeding
           it from a breadth-first spanning forest (closed form) and applying the other
           edges as one batch, beside the fixed-point initialisation of the same graph
  partitioned  n = 20k, m = 200k with 16 planted communities (1% of edges across them);
           one step partitions the graph (16 blocks), computes S of the blocks block by
           block and applies the cross-block edges as one batch
  topk     the batch graph (n = 50k, m = 1M) after one batch of updates; one step serves
           4,096 top-100 single-source queries from the stored S
  adjoint  n = 20k, m = 200k weighted (lognormal(0, 0.5)), dL/dw of a loss over 4,096 pairs
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
FP32_PEAK_TFLOPS = 157.3
C = 0.6
# the oracle's all-core leg uses at most this many host threads (one GPU's share of a host)
MAX_ORACLE_WORKERS = 16
ORACLE_POOL = None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="batch",
                    choices=["batch", "stream", "columns", "columns_batch", "forest",
                             "partitioned", "topk", "adjoint"])
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--m", type=int, default=None)
    ap.add_argument("--max-batch", type=int, default=4096)
    ap.add_argument("--chunk", type=int, default=0,
                    help="low-rank blocks per fused pass (0: the autotuner picks it, and the "
                         "GEMM tile variant, at the size after the warm-up; in column mode "
                         "the library's memory-bounded default)")
    ap.add_argument("--update-prec", default="fp64", choices=["fp64", "fp32"],
                    help="batch: arithmetic of the fused passes (fp32: float32 matrix cores, "
                         "sums added to the store in float64)")
    ap.add_argument("--no-graphs", action="store_true",
                    help="plain launches instead of replaying captured series chains")
    ap.add_argument("--no-fused", action="store_true")
    ap.add_argument("--no-tile-skip", action="store_true",
                    help="fused passes run every k-step of every tile (the same S bit for bit)")
    ap.add_argument("--split-rows", type=int, default=0,
                    help="graph rows above this many entries are traversed in chunks "
                         "(0: the library default)")
    ap.add_argument("--plain-edges", type=int, default=24)
    ap.add_argument("--store", default="blocks", choices=["blocks", "dense"],
                    help="partitioned: S per pair of partition blocks (Example 1.1), or one "
                         "dense n x n store")
    ap.add_argument("--p-cross", type=float, default=0.01,
                    help="partitioned: fraction of planted cross-community edges")
    ap.add_argument("--parts", type=int, default=16, help="partitioned: blocks")
    ap.add_argument("--partition", default="bfs", choices=["bfs", "planted"],
                    help="partitioned: the library's breadth-first partitioner, or the "
                         "planted communities (standing in for a partitioner that finds them)")
    ap.add_argument("--case-edges", type=int, default=4,
                    help="single edges timed per case C0-C3 on the plain path")
    ap.add_argument("--cb-edges", default="48,16,16",
                    help="columns_batch: insertions, deletions, insertions sharing one sink")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--fp64-shadow", action="store_true",
                    help="batch: replay the same batches on a float64 store afterwards "
                         "(untimed) and report the store's gap on sampled rows")
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
    global ORACLE_POOL
    if not args.no_cpu_baseline:
        # the oracle's worker processes start before this process touches the GPU
        ORACLE_POOL = OraclePool(min(len(os.sched_getaffinity(0)), MAX_ORACLE_WORKERS))
    import torch
    torch.cuda.set_device(0)
    run = {"batch": run_batch, "stream": run_stream, "columns": run_columns,
           "columns_batch": run_columns_batch, "forest": run_forest,
           "partitioned": run_partitioned, "topk": run_topk,
           "adjoint": run_adjoint}[args.workload]
    out = run(args)
    if ORACLE_POOL is not None:
        ORACLE_POOL.close()
    print(json.dumps(out), flush=True)


def common(args, cfg, value, unit, dt, steps, dtype="f64", extra_cfg=None):
    c = {"workload": cfg["name"], "n": args.n or cfg["n"], "m": args.m or cfg["m"],
         "C": cfg["C"], "K": cfg["K"], "parallelism": "single GPU", "steps": steps,
         "warmup": args.warmup}
    c.update(extra_cfg or {})
    return {"metric": METRIC, "value": value, "unit": unit, "n_gpus": 1, "steps": steps,
            "warmup": args.warmup, "ms_per_step": 1e3 * dt / max(steps, 1),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
            "data": "synthetic", "config": c}


def counters_for(args, name):
    """The configuration under which committed HBM counters apply: the workload name with the
    run's steps and warmup (the graph and S grow from step to step, so counters taken on
    another run length describe another state); none for resized runs."""
    if args.n or args.m:
        return "resized"
    return f"{name} steps={args.steps} warmup={args.warmup}"


def hbm_roof(bytes_, ms, kernel, launches, algorithmic, workload):
    gbs = bytes_ / (ms / 1e3) / 1e9
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic(kernel, workload),
            "kernel": kernel,
            "launches": launches, "avg_ms": round(ms / max(launches, 1), 3),
            "algorithmic": algorithmic}


# ------------------------------------------------------------------------------ batch
def run_batch(args):
    import numpy as np
    import torch

    import workloads as W
    from paper_1711_00121_amd import Context

    cfg = W.WORKLOADS[3]
    n, m, K = args.n or cfg["n"], args.m or cfg["m"], cfg["K"]
    nb = args.warmup + args.steps + 1
    log(f"bench: generating Chung-Lu n={n} m={m} and {nb} batches")
    s, d = W.chung_lu(n, m, seed=1003)
    batches, counts = W.batch_stream(n, s, d, nb, args.max_batch, seed=2003)
    t0 = time.perf_counter()
    ctx = Context(n, s, d, C=C, K=K, s_prec="hilo", node_cap=counts[-1] + 64,
                  split_rows=args.split_rows,
                  edge_cap=m + sum(len(b[0]) for b in batches) + 1024,
                  fused_batch=not args.no_fused, batch_chunk=args.chunk or 64,
                  graphs=not args.no_graphs, update_prec=args.update_prec,
                  tile_skip=not args.no_tile_skip)
    torch.cuda.synchronize()
    log(f"bench: init (S by fixed point on device) {time.perf_counter() - t0:.1f}s")

    for w in range(args.warmup):
        bi, bj, bo = batches[w]
        ctx.apply_batch(bi, bj, bo)
        torch.cuda.synchronize()
        log(f"bench: warmup batch {w} ({len(bi)} edges) done")

    tuning = None
    if args.chunk == 0 and not args.no_fused:
        t1 = time.perf_counter()
        tuning = ctx.tune()
        tuning["seconds"] = round(time.perf_counter() - t1, 2)
        log(f"bench: autotuned batch_chunk={tuning['batch_chunk']} "
            f"variant={tuning['variant']} ({'cached' if tuning['cached'] else 'measured'})")
    chunk = ctx.cfg.batch_chunk
    n_first = ctx.sizes()[0]
    ctx.profile(True)
    ctx.profile_read(reset=True)
    edges_in = edges_net = pairs = lowrank = passes = replays = 0
    flops = dense_flops = 0.0
    # net edges per Table 2 case (C0 insertions and deletions apart), from the batch plans
    mix = {"C0+": 0, "C0-": 0, "C1": 0, "C2": 0, "C3": 0}
    plan_s = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        bi, bj, bo = batches[args.warmup + k]
        st = ctx.apply_batch(bi, bj, bo, stats=True)
        tp = time.perf_counter()
        for b in ctx.last_plan():
            key = ("C0+" if b["op"] > 0 else "C0-") if b["case"] == 0 else f"C{b['case']}"
            mix[key] += len(b["I"])
        plan_s += time.perf_counter() - tp
        edges_in += len(bi)
        edges_net += st["edges_net"]
        pairs += st["pairs"]
        lowrank += st["lowrank_blocks"]
        passes += st["fused_passes"]
        replays += st["series_replays"]
        nt = float(st["n_after"])
        # Delta S is symmetric: a fused pass's work is, per low-rank block, the distinct
        # entries (a <= b) over the nodes the pass reaches, at 2 (K + 1) multiply-adds each,
        # less the k-steps (4 multiply-adds per entry) that tiles skip where the block's xi
        # factors vanish; without fused passes a block covers all n (n + 1) / 2
        if st["fused_passes"]:
            flops += float(st["pass_entries"]) * 4 * (K + 1) - 8.0 * st["pass_skipped"]
            dense_flops += float(st["pass_entries"]) * 4 * (K + 1)
        else:
            flops += nt * (nt + 1.0) * 2 * (K + 1) * st["lowrank_blocks"]
        log(f"bench: step {k}: {len(bi)} edges ({st['edges_net']} net), {st['blocks']} blocks "
            f"({st['lowrank_blocks']} low-rank), {st['fused_passes']} fused passes, "
            f"n = {st['n_after']}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0 - plan_s  # the plan copies are bookkeeping, not timed
    kern_ms, launches = ctx.profile_read(reset=True)
    ctx.profile(False)
    n_last, m_last = ctx.sizes()
    assert sum(mix.values()) == edges_net

    # Accuracy of the timed state: stored rows against the oracle's converged columns of the
    # graph after the timed batches (the hub, the newest node, sinks of the last batch, and
    # two uniform nodes), and exact symmetry of sampled entries.
    applied = list(zip(batches[:args.warmup + args.steps], counts[:args.warmup + args.steps]))
    fn, fs, fd = graph_after(n, s, d, applied)
    assert fn == n_last and len(fs) == m_last
    accuracy = None
    if ORACLE_POOL is not None:
        indeg = np.bincount(np.asarray(fd), minlength=fn)
        last_sinks = list(dict.fromkeys(int(x) for x in batches[args.warmup + args.steps - 1][1]))
        g = np.random.default_rng(11)
        xs = list(dict.fromkeys([int(np.argmax(indeg)), fn - 1] + last_sinks[:4] +
                                [int(x) for x in g.integers(fn, size=2)]))
        exact = oracle_columns(fn, fs, fd, xs)
        got = np.stack([ctx.query_column(x).cpu().numpy() for x in xs])
        pa = g.integers(fn, size=200000).astype(np.int32)
        pb = g.integers(fn, size=200000).astype(np.int32)
        sym = int((ctx.gather_pairs(pa, pb) != ctx.gather_pairs(pb, pa)).sum())
        accuracy = {"vs": "oracle FP64 converged single-source columns of the graph after the "
                          "timed batches (tail <= 1e-13)",
                    "nodes": xs, "max_abs": float(np.abs(got - exact).max()),
                    "bar": 1e-6, "asymmetric_pairs_of_200000": sym}
        log(f"bench: accuracy of the timed state {accuracy['max_abs']:.2e} on {len(xs)} columns")

    if args.fp64_shadow:
        # the same batches on a float64 store: the value + compensation store's gap from it
        g = np.random.default_rng(13)
        rows = list(dict.fromkeys((accuracy["nodes"] if accuracy else []) +
                                  [int(x) for x in g.integers(n_last, size=56)]))
        got = torch.stack([ctx.query_column(x) for x in rows])
        ref = Context(n, s, d, C=C, K=K, s_prec="fp64", node_cap=counts[-1] + 64,
                      update_prec="fp64",
                      split_rows=args.split_rows,
                      edge_cap=m + sum(len(b[0]) for b in batches) + 1024,
                      fused_batch=not args.no_fused, batch_chunk=chunk,
                      graphs=not args.no_graphs)
        ref.set_tuning(chunk, 0)
        for t in range(args.warmup + args.steps):
            ref.apply_batch(*batches[t])
            log(f"bench: float64-store replay, batch {t} done")
        gap = float((got - torch.stack([ref.query_column(x) for x in rows])).abs().max())
        ref.close()
        del got
        torch.cuda.empty_cache()
        accuracy = dict(accuracy or {})
        accuracy.update({"store_gap_vs_fp64_store": gap, "store_gap_rows": len(rows)})
        log(f"bench: store gap vs float64 store {gap:.2e} on {len(rows)} rows")

    # Plain GPU path: one apply_edge_update per edge on the same state and precision, per
    # Table 2 case: single edges into a new sink (C1), from a new source (C2) and between two
    # new nodes (C3), then C0 insertions and deletions from the next batch (edges whose net
    # effect in it is that single operation, all between nodes that existed before). The
    # batched path is compared with these per-case times weighted by the timed batches' own
    # case mix.
    from collections import Counter
    bi, bj, bo = batches[args.warmup + args.steps]
    cnt = Counter((int(a), int(b)) for a, b in zip(bi, bj))
    ins, dels = [], []
    for a, b, o in zip(bi.tolist(), bj.tolist(), bo.tolist()):
        if a < n_last and b < n_last and cnt[(a, b)] == 1:
            (ins if o > 0 else dels).append((a, b, o))
    sample = ins[:args.plain_edges] + dels[:args.plain_edges // 2]
    times = {"C0+": [], "C0-": []}
    for case in ("C1", "C2", "C3"):
        times[case] = []
        rng = np.random.default_rng(4203)
        for _ in range(args.case_edges):
            n_cur = ctx.sizes()[0]
            if case == "C1":
                a, b = int(rng.integers(n_cur)), n_cur
            elif case == "C2":
                a, b = n_cur, int(rng.integers(n_cur))
            else:
                a, b = n_cur, n_cur + 1
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            ctx.apply_edge_update(a, b, 1)
            torch.cuda.synchronize()
            times[case].append(time.perf_counter() - t1)
    # the C0 edges last, so that their streaming-kernel launches end the run's launches of it
    # (profiles pick them as the last ones)
    ctx.profile(True)
    plain_pairs = 0
    for a, b, o in sample:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        plain_pairs += ctx.apply_edge_update(a, b, o, stats=True)["pairs"]
        times["C0+" if o > 0 else "C0-"].append(time.perf_counter() - t1)
    plain_ms, plain_launches = ctx.profile_read(reset=True)
    ctx.profile(False)
    per_case = {c: (1e3 * float(np.mean(v)) if v else None) for c, v in times.items()}
    weighted = sum(mix[c] * per_case[c] for c in mix if mix[c]) / max(edges_net, 1) \
        if all(per_case[c] is not None for c in mix if mix[c]) else None
    plain_rate = 1e3 / weighted if weighted else None
    edge_rate = edges_net / dt

    if passes:
        achieved = flops / (kern_ms / 1e3) / 1e12
        peak = FP32_PEAK_TFLOPS if args.update_prec == "fp32" else FP64_PEAK_TFLOPS
        roof = {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak,
                "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
                "traffic": traffic("lowrank_gemm_kernel", counters_for(args, cfg["name"])),
                "kernel": "lowrank_gemm_kernel (fused batch pass)" if args.update_prec == "fp64"
                          else "lowrank_gemm_f32_kernel (fused batch pass, float32 matrix cores)",
                "launches": launches, "avg_ms": round(kern_ms / max(launches, 1), 3),
                "algorithmic": "r (r + 1) / 2 distinct entries x 4 (K + 1) flop per low-rank "
                               "block, r the nodes its fused pass reaches (nonzero panel "
                               "rows), less 8 flop per entry of each k-step a tile skips "
                               "(the block's xi factors vanish on both of its row ranges)",
                "skipped_fraction": round(1.0 - flops / dense_flops, 4) if dense_flops else 0.0}
    else:
        roof = hbm_roof(16.0 * pairs, kern_ms, "lowrank_strip_kernel", launches,
                        "16 B per pair-update (S value + compensation, read + write)",
                        counters_for(args, cfg["name"]))
    plain_roof = None
    if sample:
        plain_roof = hbm_roof(16.0 * plain_pairs, plain_ms, "lowrank_strip_kernel",
                              plain_launches,
                              "16 B per pair-update (S value + compensation, read + write)",
                              counters_for(args, cfg["name"] + "_plain"))
    cpu = None
    if ORACLE_POOL is not None:
        cpu = cpu_baseline_columns(fn, fs, fd, args.cpu_seconds,
                                   "the graph after the timed batches")
    out = common(args, cfg, pairs / dt, "pair-updates/s", dt, args.steps,
                 dtype="f64" if args.update_prec == "fp64" else "f32 fused passes, f64 series",
                 extra_cfg={"s_store": "f32 value + f32 compensation",
                            "max_batch": args.max_batch, "batch_chunk": chunk,
                            "gemm_variant": tuning["variant"] if tuning else 0,
                            "graphs": not args.no_graphs, "update_prec": args.update_prec,
                            "fused": not args.no_fused, "tile_skip": not args.no_tile_skip,
                            "n_first": n_first, "n_last": n_last,
                            "m_last": m_last})
    out.update({
        "edge_updates_per_s": edge_rate, "edges_net": edges_net, "edges_in": edges_in,
        "edges_in_per_s": edges_in / dt, "net_edges_by_case": mix,
        "lowrank_blocks": lowrank, "fused_passes": passes, "series_graph_replays": replays,
        "tuning": tuning,
        "plain_gpu": {"ms_per_edge_by_case": per_case,
                      "edges_timed_by_case": {c: len(v) for c, v in times.items()},
                      "ms_per_edge_at_batch_mix": weighted,
                      "edge_updates_per_s": plain_rate,
                      "c0_pair_updates_per_s": (plain_pairs / (sum(times["C0+"]) +
                                                               sum(times["C0-"])))
                      if sample else None,
                      "roofline": plain_roof},
        "speedup_edges_vs_plain": (edge_rate / plain_rate) if plain_rate else None,
        "roofline": roof,
        "accuracy": accuracy,
        "hbm_rmw_ceiling_gbs": rmw_ceiling(8.0 * n_last * n_last),
        "cpu_baseline": cpu,
    })
    return out


# ------------------------------------------------------------------------------ stream
def run_stream(args):
    import torch

    import workloads as W
    from paper_1711_00121_amd import Context

    cfg = W.WORKLOADS[2]
    n, m, K = args.n or cfg["n"], args.m or cfg["m"], cfg["K"]
    log(f"bench: generating Chung-Lu n={n} m={m} and {cfg['updates']} updates")
    s, d = W.chung_lu(n, m, seed=1002)
    oi, oj, oo = W.mixed_stream(n, s, d, cfg["updates"], cfg["p_insert"], seed=2002)
    ctx = Context(n, s, d, C=C, K=K, s_prec="hilo", prune=True)
    torch.cuda.synchronize()
    stream = list(zip(oi.tolist(), oj.tolist(), oo.tolist()))
    wu = min(args.warmup * 10, len(stream) // 10)
    for i, j, op in stream[:wu]:
        ctx.apply_edge_update(i, j, op)
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_read(reset=True)
    pairs = 0
    t0 = time.perf_counter()
    for t, (i, j, op) in enumerate(stream[wu:]):
        pairs += ctx.apply_edge_update(i, j, op, stats=True)["pairs"]
        if (t + 1) % 250 == 0:
            log(f"bench: {t + 1} updates")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kern_ms, launches = ctx.profile_read(reset=True)
    ctx.profile(False)
    done = len(stream) - wu
    out = common(args, cfg, pairs / dt, "pair-updates/s", dt, done,
                 extra_cfg={"s_store": "f32 value + f32 compensation", "prune": True,
                            "updates": done, "p_insert": cfg["p_insert"]})
    out["edge_updates_per_s"] = done / dt
    out["mean_pairs_per_update"] = pairs / done
    out["roofline"] = hbm_roof(16.0 * pairs, kern_ms, "lowrank_strip_kernel", launches,
                               "16 B per pair-update (S value + compensation, read + write)",
                               counters_for(args, cfg["name"]))
    out["hbm_rmw_ceiling_gbs"] = rmw_ceiling(8.0 * n * n)
    # Precision: the same stream on a float64 store (untimed), and both against the
    # oracle's converged columns of the final graph at sampled nodes.
    ref = Context(n, s, d, C=C, K=K, s_prec="fp64", prune=True)
    for i, j, op in stream:
        ref.apply_edge_update(i, j, op)
    torch.cuda.synchronize()
    S_hilo = ctx.S()
    gap = float((S_hilo - ref.S()).abs().max())
    del S_hilo
    torch.cuda.empty_cache()
    fs, fd = final_edges(s, d, stream)
    out["accuracy"] = {"store_gap_vs_fp64_store": gap}
    if not args.no_cpu_baseline:
        import numpy as np
        indeg = np.bincount(fd, minlength=n)
        xs = list(dict.fromkeys([int(np.argmax(indeg))] + [int(x) for x in stream[-1][:2]] +
                                [int(x) for x in np.random.default_rng(12).integers(n, size=5)]))
        exact = oracle_columns(n, fs, fd, xs)
        got = np.stack([ctx.query_column(x).cpu().numpy() for x in xs])
        got64 = np.stack([ref.query_column(x).cpu().numpy() for x in xs])
        out["accuracy"].update({
            "vs": "oracle FP64 converged single-source columns of the final graph",
            "nodes": xs, "max_abs": float(np.abs(got - exact).max()),
            "max_abs_fp64_store": float(np.abs(got64 - exact).max()), "bar": 1e-6})
    ref.close()
    out["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_columns(n, fs, fd, args.cpu_seconds,
                                                   "the graph after the stream")
    return out


# ------------------------------------------------------------------------------ columns
def run_columns(args):
    import torch

    import workloads as W
    from paper_1711_00121_amd import Context

    cfg = W.WORKLOADS[4]
    n, m, K, Kps = args.n or cfg["n"], args.m or cfg["m"], cfg["K"], cfg["K_ps"]
    steps = args.steps
    log(f"bench: generating Chung-Lu n={n} m={m}")
    s, d = W.chung_lu(n, m, seed=1004)
    ii, jj = W.insertion_stream(n, s, d, args.warmup + steps, seed=2004)
    cols = W.column_sample(n, cfg["columns"], seed=3004)[:cfg["columns"]]
    blocks = [cols[b:b + cfg["block"]] for b in range(0, len(cols), cfg["block"])]
    ctx = Context(n, s, d, C=C, K=K, K_ps=Kps, mode="column",
                  edge_cap=m + args.warmup + steps + 1024, split_rows=args.split_rows)
    out_buf = torch.empty((cfg["block"], n), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()

    def one(t):
        ctx.apply_edge_update(int(ii[t]), int(jj[t]), 1)
        for blk in blocks:
            ctx.query_columns(blk, out=out_buf[:len(blk)])

    for t in range(args.warmup):
        one(t)
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_read(reset=True)
    t0 = time.perf_counter()
    for t in range(args.warmup, args.warmup + steps):
        one(t)
        log(f"bench: insertion {t - args.warmup + 1}/{steps}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kern_ms, launches = ctx.profile_read(reset=True)
    ctx.profile(False)
    # precision of the float32 output: the last block's first columns against the float64
    # Delta S columns of the same (last) insertion
    last = blocks[-1][:8]
    got = out_buf[:len(last)].double()
    ref64 = torch.stack([ctx.query_column(int(x), what="delta") for x in last])
    out32_gap = float((got - ref64).abs().max())
    out32_scale = float(ref64.abs().max())
    del got, ref64
    values = float(n) * len(cols) * steps
    out = common(args, cfg, values / dt, "pair-values/s", dt, steps,
                 extra_cfg={"K_ps": Kps, "columns": len(cols), "block": cfg["block"],
                            "output": "float32"})
    out["accuracy"] = {"vs": "float64 Delta S columns of the same insertion (query_column)",
                       "columns": len(last), "max_abs_float32_output_vs_fp64": out32_gap,
                       "max_abs_delta": out32_scale,
                       "note": "float64 arithmetic; only the output is rounded to float32"}
    out["metric"] = "ΔS column values/s, column-by-column mode (no stored S)"
    out["columns_per_s"] = len(cols) * steps / dt
    # each output value is a 2 (K + 1)-term dot product (4 (K + 1) flop) written as 4 bytes;
    # at the peaks the flops take longer than the writes, so the kernel is bound by FP64 MFMA
    flops = 4.0 * (K + 1) * values
    achieved = flops / (kern_ms / 1e3) / 1e12
    out["roofline"] = {"bound": "mfma", "achieved": round(achieved, 2),
                       "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                       "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
                       "traffic": traffic("lowrank_cols_kernel", counters_for(args, cfg["name"])),
                       "kernel": "lowrank_cols_kernel", "launches": launches,
                       "avg_ms": round(kern_ms / max(launches, 1), 3),
                       "algorithmic": "4 (K + 1) flop and 4 B written per output value",
                       "write_gbs": round(4.0 * values / (kern_ms / 1e3) / 1e9, 1)}
    out["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_delta_columns(n, s, d, int(ii[0]), int(jj[0]), cols,
                                                         K, Kps, args.cpu_seconds)
    return out


# ------------------------------------------------------------------------------ columns_batch
def run_columns_batch(args):
    import torch

    import workloads as W
    from paper_1711_00121_amd import Context

    cfg = W.WORKLOADS[4]
    n, m, K, Kps = args.n or cfg["n"], args.m or cfg["m"], cfg["K"], cfg["K_ps"]
    n_ins, n_del, shared = (int(x) for x in args.cb_edges.split(","))
    steps = args.steps
    log(f"bench: generating Chung-Lu n={n} m={m}")
    s, d = W.chung_lu(n, m, seed=1004)
    batches = W.existing_batches(n, s, d, args.warmup + steps, n_ins, n_del, shared, seed=2204)
    cols = W.column_sample(n, cfg["block"], seed=3004)[:cfg["block"]]
    from paper_1711_00121_amd import device_bytes
    held_before, _ = device_bytes()
    ctx = Context(n, s, d, C=C, K=K, K_ps=Kps, mode="column",
                  edge_cap=m + (args.warmup + steps) * n_ins + 1024,
                  split_rows=args.split_rows, batch_chunk=args.chunk)
    chunk = ctx.config().batch_chunk
    held_ctx, _ = device_bytes(reset_peak=True)
    out_buf = torch.empty((len(cols), n), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    for t in range(args.warmup):
        ctx.apply_batch_columns(*batches[t], cols, out=out_buf)
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_read(reset=True)
    blocks = passes = 0
    t0 = time.perf_counter()
    for t in range(args.warmup, args.warmup + steps):
        _, st = ctx.apply_batch_columns(*batches[t], cols, out=out_buf, stats=True)
        blocks += st["blocks"]
        passes += st["fused_passes"]
        log(f"bench: batch {t - args.warmup + 1}/{steps}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kern_ms, launches = ctx.profile_read(reset=True)
    ctx.profile(False)
    _, peak = device_bytes()
    values = float(n) * len(cols) * steps
    edges = (n_ins + n_del) * steps
    out = common(args, cfg, values / dt, "pair-values/s", dt, steps,
                 extra_cfg={"workload": "column_batch_n1m", "K_ps": Kps,
                            "columns": len(cols), "batch": {"insert": n_ins, "delete": n_del,
                                                            "shared_sink": shared},
                            "output": "float64", "batch_chunk": chunk})
    # memory: what the library holds (graph, series and PartialSim buffers, the panel), not
    # the caller's output; an n x n store would be n^2 x 8 bytes
    w = 2 * (K + 1)
    out["memory"] = {"library_bytes_after_init": held_ctx - held_before,
                     "library_bytes_peak": peak - held_before,
                     "panel_bytes": -(-chunk * w // 16) * 16 * (-(-n // 128) * 128) * 8,
                     "series_bytes_Kn": 2 * (K + 1) * n * 8,
                     "output_bytes": len(cols) * n * 8,
                     "dense_S_bytes": n * n * 8}
    out["accuracy"] = {"note": "float64 arithmetic and output throughout; parity against the "
                               "oracle's column method is in the GPU tests (1e-12 relative)"}
    out["metric"] = "batch Delta S column values/s, column-by-column mode (no stored S)"
    out["edges_per_s"] = edges / dt
    out["blocks_per_batch"] = blocks / steps
    # the accumulate adds P[cols] P^T for the whole batch: 2 (K + 1) panel columns per block,
    # 2 flop per panel column and output value
    flops = 2.0 * len(cols) * n * 2 * (K + 1) * blocks
    achieved = flops / (kern_ms / 1e3) / 1e12
    out["roofline"] = {"bound": "mfma", "achieved": round(achieved, 2),
                       "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                       "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
                       "traffic": traffic("lowrank_gemm_kernel_rect", counters_for(args, "column_batch_n1m")),
                       "kernel": "lowrank_gemm_kernel (rectangular accumulate)",
                       "launches": launches, "avg_ms": round(kern_ms / max(launches, 1), 3),
                       "share_of_step": round(kern_ms / (1e3 * dt), 3),
                       "algorithmic": "2 (K + 1) panel columns per block; 2 flop per panel "
                                      "column and output value"}
    out["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_columns_batch(n, s, d, batches[0], cols[:64], K, Kps,
                                                         args.cpu_seconds)
    return out


# ------------------------------------------------------------------------------ forest
def run_forest(args):
    import numpy as np
    import torch

    import workloads as W
    from paper_1711_00121_amd import Context

    cfg = W.WORKLOADS[2]
    n, m, K = args.n or cfg["n"], args.m or cfg["m"], cfg["K"]
    log(f"bench: generating Chung-Lu n={n} m={m}")
    s, d = W.chung_lu(n, m, seed=1002)
    common_cfg = dict(C=C, K=K, s_prec="hilo", batch_chunk=args.chunk or 64,
                      split_rows=args.split_rows)

    def seeded(profile=False):
        return Context(n, s, d, init="forest", profile=profile, **common_cfg)

    for w in range(args.warmup):
        seeded().close()
        torch.cuda.synchronize()
        log(f"bench: warmup {w} done")
    times, kern_ms, launches = [], 0.0, 0
    ctx = None
    for k in range(args.steps):
        if ctx is not None:
            ctx.close()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx = seeded(profile=True)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        ms, cnt = ctx.profile_read(reset=True)
        kern_ms += ms
        launches += cnt
        log(f"bench: step {k}: {times[-1]:.2f} s, {ctx.init_stats['blocks']} blocks, "
            f"{ctx.init_stats['fused_passes']} fused passes")
    st = ctx.init_stats
    dt = float(np.sum(times))
    # the fixed-point initialisation of the same graph, and how far the two S are apart
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ref = Context(n, s, d, **common_cfg)
    torch.cuda.synchronize()
    t_fixed = time.perf_counter() - t1
    diff = float((ctx.S() - ref.S()).abs().max())
    ref.close()
    accuracy = oracle_accuracy(ctx, n, s, d, "the graph")
    out = common(args, cfg, float(n) * n * args.steps / dt, "S entries/s", dt, args.steps,
                 extra_cfg={"workload": "forest_seeded_n20k", "s_store": "f32 value + f32 "
                            "compensation", "batch_chunk": args.chunk or 64})
    out["accuracy"] = accuracy
    out["metric"] = "all-pairs SimRank seeded from a spanning forest (Example 1.2), S entries/s"
    out["seconds_per_all_pairs"] = dt / args.steps
    out["forest"] = {"tree_edges": m - st["edges_in"], "batch_edges": st["edges_in"],
                     "blocks": st["blocks"], "lowrank_blocks": st["lowrank_blocks"],
                     "fused_passes": st["fused_passes"]}
    out["fixed_point_init_s"] = t_fixed
    out["max_abs_vs_fixed_point"] = diff
    pld = 2 * (K + 1)
    flops = (float(st["pass_entries"]) * 2 * pld - 8.0 * st["pass_skipped"]) * args.steps
    achieved = flops / (kern_ms / 1e3) / 1e12
    out["roofline"] = {"bound": "mfma", "achieved": round(achieved, 2),
                       "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                       "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
                       "traffic": traffic("lowrank_gemm_kernel", counters_for(args, "forest_seeded_n20k")),
                       "kernel": "lowrank_gemm_kernel (fused batch pass)",
                       "launches": launches, "avg_ms": round(kern_ms / max(launches, 1), 3),
                       "share_of_step": round(kern_ms / (1e3 * dt), 3),
                       "algorithmic": "r (r + 1) / 2 distinct entries x 4 (K + 1) flop per "
                                      "low-rank block, r the nodes its fused pass reaches"}
    ctx.close()
    out["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_forest(K, args.cpu_seconds)
    return out


# ------------------------------------------------------------------------------ partitioned
def run_partitioned(args):
    import numpy as np
    import torch

    import workloads as W
    from paper_1711_00121_amd import Context, partition

    cfg = W.WORKLOADS[2]
    n, m, K = args.n or cfg["n"], args.m or cfg["m"], cfg["K"]
    p_cross, parts = args.p_cross, args.parts
    log(f"bench: generating {parts} planted communities n={n} m={m}")
    s, d, planted = W.communities(n, m, parts, p_cross, seed=1102)
    common_cfg = dict(C=C, K=K, s_prec="hilo", batch_chunk=args.chunk or 64,
                      split_rows=args.split_rows)
    store_cfg = dict(block_store=True) if args.store == "blocks" else {}

    def build(profile=False):
        lab = planted if args.partition == "planted" else partition(n, s, d, parts)
        return Context(n, s, d, init="partitioned", part=lab, profile=profile, **common_cfg,
                       **store_cfg)

    for w in range(args.warmup):
        build().close()
        torch.cuda.synchronize()
    times, kern_ms, launches = [], 0.0, 0
    ctx = None
    for k in range(args.steps):
        if ctx is not None:
            ctx.close()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx = build(profile=True)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        ms, cnt = ctx.profile_read(reset=True)
        kern_ms += ms
        launches += cnt
        log(f"bench: step {k}: {times[-1]:.2f} s, {ctx.init_stats['edges_in']} cross edges, "
            f"{ctx.init_stats['blocks']} blocks")
    st = ctx.init_stats
    dt = float(np.sum(times))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ref = Context(n, s, d, **common_cfg)
    torch.cuda.synchronize()
    t_fixed = time.perf_counter() - t1
    diff = float((ctx.S() - ref.S()).abs().max())
    dense_bytes = ref.store_bytes()[0]
    ref.close()
    accuracy = oracle_accuracy(ctx, n, s, d, "the graph")
    store_bytes, store_pairs = ctx.store_bytes()
    out = common(args, cfg, float(n) * n * args.steps / dt, "S entries/s", dt, args.steps,
                 extra_cfg={"workload": "partitioned_n20k", "parts": parts,
                            "planted_cross_fraction": p_cross,
                            "partition": args.partition,
                            "s_store": "f32 value + f32 compensation",
                            "store": "block pairs" if args.store == "blocks" else "dense",
                            "batch_chunk": args.chunk or 64})
    # memory of S: the store held against n^2 entries of 8 bytes (value + compensation)
    out["store"] = {"bytes": store_bytes, "block_pairs_held": store_pairs,
                    "block_pairs": parts * (parts + 1) // 2,
                    "n2_bytes": 8 * n * n, "fraction_of_n2": store_bytes / (8.0 * n * n),
                    "dense_store_bytes": dense_bytes}
    out["metric"] = ("all-pairs SimRank over a partitioned graph (Example 1.1), S entries/s")
    out["accuracy"] = accuracy
    out["seconds_per_all_pairs"] = dt / args.steps
    out["partition"] = {"cross_edges": st["edges_in"], "blocks": st["blocks"],
                        "lowrank_blocks": st["lowrank_blocks"],
                        "fused_passes": st["fused_passes"]}
    out["fixed_point_init_s"] = t_fixed
    out["max_abs_vs_fixed_point"] = diff
    pld = 2 * (K + 1)
    if args.store == "blocks":
        # entries of the reached block pairs per deferred block (both triangles), each
        # 2 (K + 1) multiply-adds for half of them (the pass writes mirrored entries once)
        flops = float(st["pairs"]) * pld * args.steps
    else:
        flops = (float(st["pass_entries"]) * 2 * pld - 8.0 * st["pass_skipped"]) * args.steps
    achieved = flops / (kern_ms / 1e3) / 1e12 if kern_ms > 0 else 0.0
    out["roofline"] = {"bound": "mfma", "achieved": round(achieved, 2),
                       "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                       "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
                       "traffic": None if args.store == "blocks" else
                       traffic("lowrank_gemm_kernel", counters_for(args, "partitioned_n20k")),
                       "kernel": "lowrank_gemm_kernel (fused batch pass"
                                 + (", block-store mode)" if args.store == "blocks" else ")"),
                       "launches": launches, "avg_ms": round(kern_ms / max(launches, 1), 3),
                       "share_of_step": round(kern_ms / (1e3 * dt), 3),
                       "algorithmic": "r (r + 1) / 2 distinct entries x 4 (K + 1) flop per "
                                      "low-rank block, r the nodes its fused pass reaches"}
    ctx.close()
    out["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_partitioned(K, parts, p_cross, args.cpu_seconds)
    return out


# ------------------------------------------------------------------------------ topk
def run_topk(args, nq=4096, k=100):
    import numpy as np
    import torch

    import workloads as W
    from paper_1711_00121_amd import Context

    cfg = W.WORKLOADS[3]
    n, m, K = args.n or cfg["n"], args.m or cfg["m"], cfg["K"]
    log(f"bench: generating Chung-Lu n={n} m={m}")
    s, d = W.chung_lu(n, m, seed=1003)
    batches, counts = W.batch_stream(n, s, d, 1, args.max_batch, seed=2003)
    ctx = Context(n, s, d, C=C, K=K, s_prec="hilo", node_cap=counts[-1] + 64,
                  edge_cap=m + len(batches[0][0]) + 1024, batch_chunk=args.chunk or 64,
                  split_rows=args.split_rows)
    ctx.apply_batch(*batches[0])
    n_now = ctx.sizes()[0]
    torch.cuda.synchronize()
    log(f"bench: S ready after one batch, n = {n_now}")
    steps = args.steps + args.warmup
    qs = [W.rng(5003 + t).choice(n_now, nq, replace=False).astype(np.int32) for t in range(steps)]
    out_buf = (torch.empty((nq, k), dtype=torch.int32, device="cuda"),
               torch.empty((nq, k), dtype=torch.float64, device="cuda"))
    for t in range(args.warmup):
        ctx.query_topk(qs[t], k, out=out_buf)
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_read(reset=True)
    t0 = time.perf_counter()
    for t in range(args.warmup, steps):
        ctx.query_topk(qs[t], k, out=out_buf)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kern_ms, launches = ctx.profile_read(reset=True)
    ctx.profile(False)
    res = common(args, cfg, nq * args.steps / dt, "queries/s", dt, args.steps,
                 extra_cfg={"workload": "topk_serving_n50k", "queries": nq, "k": k,
                            "s_store": "f32 value + f32 compensation",
                            "after": f"one batch of {len(batches[0][0])} edge updates"})
    res["metric"] = "top-k single-source queries/s from the stored S after updates"
    # each query reads its row of the store once: n entries of 8 B (value + compensation)
    res["roofline"] = hbm_roof(8.0 * n_now * nq * args.steps, kern_ms, "topk_wave_kernel",
                               launches, "one row of the store per query (8 B per entry)",
                               counters_for(args, "topk_serving_n50k"))
    res["accuracy"] = None
    if ORACLE_POOL is not None:
        # served lists against the oracle's converged columns of the graph after the batch:
        # precision@k of the sets and the largest error of a served value
        fn, fs, fd = graph_after(n, s, d, [(batches[0], counts[0])])
        qx = [int(x) for x in qs[-1][:8]]
        exact = oracle_columns(fn, fs, fd, qx)
        idx, val = ctx.query_topk(np.asarray(qx, np.int32), k)
        idx, val = idx.cpu().numpy(), val.cpu().numpy()
        prec, err = [], 0.0
        for t, x in enumerate(qx):
            col = exact[t].copy()
            col[x] = -np.inf  # the query itself is excluded
            best = np.argsort(-col, kind="stable")[:k]
            prec.append(len(set(best.tolist()) & set(idx[t].tolist())) / k)
            err = max(err, float(np.abs(val[t] - exact[t][idx[t]]).max()))
        res["accuracy"] = {"vs": "oracle FP64 converged columns of the graph after the batch",
                           "queries": qx, "precision_at_k_min": min(prec),
                           "precision_at_k_mean": float(np.mean(prec)),
                           "max_abs_served_value": err}
    res["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        rows = np.stack([ctx.query_column(int(x)).cpu().numpy() for x in qs[0][:256]])
        res["cpu_baseline"] = cpu_baseline_topk(rows, qs[0][:256], k, args.cpu_seconds)
    ctx.close()
    return res


# ------------------------------------------------------------------------------ adjoint
def run_adjoint(args):
    import torch

    import workloads as W
    from paper_1711_00121_amd import Context

    cfg = W.WORKLOADS[5]
    n, m, K = args.n or cfg["n"], args.m or cfg["m"], cfg["K"]
    log(f"bench: generating weighted Chung-Lu n={n} m={m}")
    s, d = W.chung_lu(n, m, seed=1005)
    w = W.lognormal_weights(m, seed=3005)
    a, b, tgt = W.loss_pairs(n, cfg["pairs"], seed=3105)
    ctx = Context(n, s, d, weight=w, C=C, K=K, s_prec="fp64")
    at = torch.as_tensor(a, device="cuda")
    bt = torch.as_tensor(b, device="cuda")
    tt = torch.as_tensor(tgt, device="cuda")

    def step():
        vals = ctx.gather_pairs(at, bt)
        return ctx.backward(at, bt, 2.0 * (vals - tt))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_read(reset=True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kern_ms, launches = ctx.profile_read(reset=True)
    ctx.profile(False)
    # Plain path to the same gradient: one incremental unit update per edge (its first-order
    # part is the directional derivative), timed on a few insertions into an unweighted
    # context of the same graph at the same accuracy.
    plain = Context(n, s, d, C=C, K=K, s_prec="fp64", prune=True)
    ins_i, ins_j = W.insertion_stream(n, s, d, 8, seed=3405)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for i, j in zip(ins_i.tolist(), ins_j.tolist()):
        plain.apply_edge_update(i, j, 1)
    torch.cuda.synchronize()
    per_edge = (time.perf_counter() - t1) / len(ins_i)
    out = common(args, cfg, m * args.steps / dt, "edge-gradients/s", dt, args.steps,
                 extra_cfg={"pairs": cfg["pairs"], "weights": "lognormal(0, 0.5)"})
    out["metric"] = "dL/dw for all m edge weights per second (adjoint of eq (03a))"
    out["plain_gpu"] = {"seconds_per_edge_update": per_edge,
                        "seconds_for_all_edges": per_edge * m,
                        "speedup_adjoint_vs_plain": per_edge * m / (dt / args.steps)}
    # spmm_qt_rows: reads X and writes Y (n^2 float64 each); the second product of an
    # iteration also reads G and the previous iterate
    nbytes = 8.0 * n * n * 3.0 * launches
    out["roofline"] = hbm_roof(nbytes, kern_ms, "spmm_qt_rows_kernel", launches,
                               "n^2 x 8 B read + n^2 x 8 B written (+ 2 n^2 x 8 B read on "
                               "every second launch)", counters_for(args, cfg["name"]))
    out["accuracy"] = None
    out["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        import numpy as np
        # dL/dw for unit upstream gradients at the pairs, on 16 edges, against the oracle's
        # per-edge adjoint form (converged columns, no dense matrices)
        edges = np.sort(W.rng(3305).choice(m, 16, replace=False))
        dw = ctx.backward(at, bt, torch.ones(len(a), dtype=torch.float64,
                                             device="cuda")).cpu().numpy()
        path = ORACLE_POOL.stage(n=n, s=np.asarray(s, np.int64), d=np.asarray(d, np.int64),
                                 w=w, a=a, b=b, C=C)
        ref = np.asarray(ORACLE_POOL.map("gradient", path, [int(e) for e in edges]))
        out["accuracy"] = {"vs": "oracle FP64 per-edge adjoint (converged columns)",
                           "edges": len(edges), "max_abs": float(np.abs(dw[edges] - ref).max()),
                           "max_abs_gradient": float(np.abs(ref).max())}
        out["cpu_baseline"] = cpu_baseline_gradient(n, s, d, w, a, b, args.cpu_seconds)
    return out


# ------------------------------------------------------------------------------ helpers
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


def rmw_ceiling(nbytes):
    """Read-modify-write bandwidth of a plain library kernel (torch's in-place add) over a
    buffer of `nbytes` (the size of the stored S): the practical ceiling of an update that
    reads and writes every entry once at that footprint, beside the 8 TB/s peak. (Smaller
    footprints run faster: about 5.8 TB/s at 2 GB against 5.4 TB/s at 26 GB.)"""
    import torch
    x = torch.zeros(int(nbytes) // 8, dtype=torch.float64, device="cuda")
    x.add_(1.0)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        x.add_(1.0)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    gbs = 3 * 2 * x.numel() * 8 / (ms / 1e3) / 1e9
    del x
    torch.cuda.empty_cache()
    return round(gbs, 1)


def traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed counter summary, or None when the
    counters were taken on another workload or run configuration (steps, warmup), or the
    kernel's source has changed since."""
    import hashlib
    import re
    name = kernel.split(" ")[0]
    path = os.path.join(ROOT, "profiles", f"{name}_{workload.split(' ')[0]}_pmc.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_src = re.search(r"Source: `([^`]+)`", text)
    m_sha = re.search(r"source_sha256:\s*([0-9a-f]{64})", text)
    # one section per run configuration: the bytes line, then its workload line
    found = dict((w.strip(), float(b)) for b, w in re.findall(
        r"^hbm_bytes_per_launch:\s*([0-9.eE+]+)\s*\nworkload:\s*(.+?)\s*$", text, flags=re.M))
    if not (m_src and m_sha) or workload not in found:
        return None
    src = os.path.join(ROOT, m_src.group(1))
    if not os.path.exists(src):
        return None
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != m_sha.group(1):
        return None
    return found[workload]


def host_cpu():
    """The host CPU the oracle runs on: model name and logical CPU counts."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(),
            "usable_cpus": len(os.sched_getaffinity(0))}


_ORACLE_STATE = {}


def _oracle_state(kind, path):
    """Per-worker state of an oracle task kind, loaded once from the npz at `path`."""
    import numpy as np
    key = (kind, path)
    if key in _ORACLE_STATE:
        return _ORACLE_STATE[key]
    z = dict(np.load(path, allow_pickle=False))
    if kind in ("columns", "delta_columns"):
        from oracle import graph as Gr
        n = int(z["n"])
        z["Q"] = Gr.transition_matrix(n, z["s"], z["d"])
    _ORACLE_STATE.clear()
    _ORACLE_STATE[key] = z
    return z


def oracle_task(kind, path, arg):
    """One unit of oracle work (runs in a worker process, one BLAS thread)."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        if kind == "warm":  # load the inputs of task kind `arg`
            _oracle_state(arg, path)
            time.sleep(0.2)  # so that every worker takes one
            return None
        z = _oracle_state(kind, path)
        if kind == "columns":
            from oracle import simrank as O
            return O.single_source(z["Q"], int(arg), float(z["C"]), tol=1e-13)
        if kind == "delta_columns":
            from oracle import incremental as OI
            OI.delta_columns_c0(int(z["n"]), z["s"], z["d"], int(z["i"]), int(z["j"]),
                                z["cols"][arg:arg + 8], float(z["C"]), int(z["K"]),
                                int(z["Kps"]))
            return None
        if kind == "gradient":
            from oracle import adjoint as OA
            return float(OA.grad_weight_edges(int(z["n"]), z["s"], z["d"], z["w"], z["a"],
                                              z["b"], None, float(z["C"]), [int(arg)],
                                              g_pairs=np.ones(len(z["a"])))[0])
        if kind == "topk":
            from oracle import serving as Sv
            r = int(arg) % len(z["q"])
            Sv.topk(z["rows"][r], int(z["q"][r]), int(z["k"]))
            return None
        if kind == "forest":
            from oracle import tree as OT
            OT.tree_seeded(int(z["n"]), z["s"], z["d"], float(z["C"]), int(z["K"]))
            return None
        if kind == "partitioned":
            from oracle import partition as OP
            lab = OP.bfs_partition(int(z["n"]), z["s"], z["d"], int(z["parts"]))
            OP.partitioned(int(z["n"]), z["s"], z["d"], lab, float(z["C"]), int(z["K"]))
            return None
    raise ValueError(kind)


class OraclePool:
    """Worker processes for the oracle's all-core leg. They are spawned before the benchmark
    touches the GPU; each task's inputs travel as an npz file that a worker loads once."""

    def __init__(self, workers):
        import multiprocessing as mp
        import tempfile
        self.workers = max(1, int(workers))
        self.pool = mp.get_context("spawn").Pool(self.workers)
        self.dir = tempfile.mkdtemp(prefix="oracle_")
        self.files = 0

    def stage(self, **arrays):
        import numpy as np
        path = os.path.join(self.dir, f"in{self.files}.npz")
        self.files += 1
        np.savez(path, **{k: np.asarray(v) for k, v in arrays.items()})
        return path

    def map(self, kind, path, args):
        """Runs the tasks to completion (untimed) and returns their results in order."""
        return self.pool.starmap(oracle_task, [(kind, path, a) for a in args])

    def rate(self, kind, path, args, seconds):
        """Runs tasks from `args` (cycled) on every worker until `seconds` have passed;
        returns (tasks done, wall seconds). Loading the inputs is not timed."""
        # every worker loads the inputs once, untimed
        self.pool.starmap(oracle_task, [("warm", path, kind)] * self.workers, chunksize=1)
        t0 = time.perf_counter()
        pending, done, t = [], 0, 0
        while True:
            while len(pending) < 2 * self.workers and time.perf_counter() - t0 < seconds:
                pending.append(self.pool.apply_async(oracle_task,
                                                     (kind, path, args[t % len(args)])))
                t += 1
            if not pending:
                break
            pending.pop(0).get()
            done += 1
        return done, time.perf_counter() - t0

    def close(self):
        import shutil
        self.pool.terminate()
        self.pool.join()
        shutil.rmtree(self.dir, ignore_errors=True)


def graph_after(n, s, d, applied):
    from oracle import graph as Gr
    from oracle import incremental as OI
    cur_n, cur_s, cur_d = n, s, d
    for (bi, bj, bo), nn in applied:
        plus, minus = OI.net_update(bi, bj, bo)
        cur_n, cur_s, cur_d = Gr.apply_edges(
            cur_n, cur_s, cur_d, [e[0] for e in plus + minus], [e[1] for e in plus + minus],
            [1] * len(plus) + [-1] * len(minus), n_new=nn)
    return cur_n, cur_s, cur_d


def final_edges(s, d, stream):
    import numpy as np
    es = set(zip(s.tolist(), d.tolist()))
    for i, j, op in stream:
        if op > 0:
            es.add((i, j))
        else:
            es.discard((i, j))
    e = sorted(es, key=lambda t: (t[1], t[0]))
    return (np.asarray([a for a, _ in e], dtype=np.int64),
            np.asarray([b for _, b in e], dtype=np.int64))


def oracle_baseline(kind, path, args, seconds, units_per_task, unit, sample):
    """The oracle timed on the host: an all-core leg (the worker pool, one thread each) and a
    one-thread leg (this process), each on a bounded number of tasks. `value` is the all-core
    rate; `cores` the worker count it used."""
    p = ORACLE_POOL
    t_all = 0.6 * seconds
    done, dt = p.rate(kind, path, args, t_all)
    from threadpoolctl import threadpool_limits
    oracle_task("warm", path, kind)
    t0 = time.perf_counter()
    done1 = 0
    with threadpool_limits(1):
        while time.perf_counter() - t0 < 0.4 * seconds:
            oracle_task(kind, path, args[done1 % len(args)])
            done1 += 1
    dt1 = time.perf_counter() - t0
    return {"value": done * units_per_task / dt, "unit": unit, "cores": p.workers,
            "kind": "oracle", "sample": f"{sample}; all-core: {done} tasks in {dt:.1f} s on "
                                        f"{p.workers} worker processes (one thread each)",
            "host": host_cpu(),
            "one_thread": {"value": done1 * units_per_task / dt1, "tasks": done1,
                           "seconds": round(dt1, 2)}}


def cpu_baseline_columns(n, s, d, seconds, what, xs=None):
    """The oracle on the host: converged single-source columns S[:, x] of the updated graph
    (eq (17) by PartialSim to a tail <= 1e-13), i.e. pair values of the updated S computed
    from scratch, timed on a bounded sample of columns (x uniform)."""
    import numpy as np
    path = ORACLE_POOL.stage(n=n, s=np.asarray(s, np.int64), d=np.asarray(d, np.int64), C=C)
    xs = list(np.random.default_rng(7).integers(n, size=512)) if xs is None else xs
    return oracle_baseline("columns", path, xs, seconds, float(n), "pair-updates/s",
                           f"converged single-source columns S[:, x] (x uniform) of {what} "
                           f"(n={n}), oracle PartialSim to a tail <= 1e-13")


def oracle_columns(n, s, d, xs):
    """Converged single-source columns of the graph at the nodes xs (all-core, untimed)."""
    import numpy as np
    path = ORACLE_POOL.stage(n=n, s=np.asarray(s, np.int64), d=np.asarray(d, np.int64), C=C)
    return np.stack(ORACLE_POOL.map("columns", path, [int(x) for x in xs]))


def oracle_accuracy(ctx, n, s, d, what):
    """Stored columns against the oracle's converged columns of the same graph (the hub and
    five uniform nodes); None when the oracle pool is off."""
    import numpy as np
    if ORACLE_POOL is None:
        return None
    indeg = np.bincount(np.asarray(d, np.int64), minlength=n)
    xs = list(dict.fromkeys([int(np.argmax(indeg))] +
                            [int(x) for x in np.random.default_rng(14).integers(n, size=5)]))
    exact = oracle_columns(n, s, d, xs)
    got = np.stack([ctx.query_column(x).cpu().numpy() for x in xs])
    return {"vs": f"oracle FP64 converged single-source columns of {what}", "nodes": xs,
            "max_abs": float(np.abs(got - exact).max()), "bar": 1e-6}


def cpu_baseline_delta_columns(n, s, d, i, j, cols, K, Kps, seconds):
    """The oracle's column-by-column Delta S (same K and PartialSim depth) for the first
    insertion, 8 columns per task."""
    import numpy as np
    path = ORACLE_POOL.stage(n=n, s=np.asarray(s, np.int64), d=np.asarray(d, np.int64), i=i,
                             j=j, cols=np.asarray(cols), C=C, K=K, Kps=Kps)
    return oracle_baseline("delta_columns", path, list(range(0, len(cols) - 8, 8)), seconds,
                           8.0 * n, "pair-values/s",
                           "Delta S columns of one insertion, 8 per oracle call")


def cpu_baseline_columns_batch(n, s, d, batch, cols, K, Kps, seconds):
    """The oracle's block-by-block Delta S columns of one batch, run on consecutive 4-edge
    slices of the batch (each on the graph the earlier slices left) until the time budget is
    used, in this process on one thread; the whole batch's time is extrapolated linearly in
    edges. (The slices depend on each other, so there is no all-core leg.)"""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import incremental as OI
    bi, bj, bo = batch
    cur_s, cur_d = s.astype(np.int64), d.astype(np.int64)
    t0 = time.perf_counter()
    done = 0
    with threadpool_limits(1):
        while time.perf_counter() - t0 < seconds and done < len(bi):
            sl = slice(done, min(done + 4, len(bi)))
            OI.delta_columns_batch(n, cur_s, cur_d, bi[sl], bj[sl], bo[sl], cols, C, K, Kps)
            ins, dels = bo[sl] > 0, bo[sl] < 0
            drop = np.isin(cur_s * n + cur_d,
                           bi[sl][dels].astype(np.int64) * n + bj[sl][dels].astype(np.int64))
            cur_s = np.concatenate([cur_s[~drop], bi[sl][ins].astype(np.int64)])
            cur_d = np.concatenate([cur_d[~drop], bj[sl][ins].astype(np.int64)])
            done = sl.stop
    dt = time.perf_counter() - t0
    per_batch = dt * len(bi) / done
    return {"value": float(n) * len(cols) / per_batch, "unit": "pair-values/s", "cores": 1,
            "kind": "oracle", "host": host_cpu(),
            "sample": f"{done} of {len(bi)} edges of one batch in 4-edge slices, "
                      f"{len(cols)} columns, {dt:.1f} s on one host thread (the slices depend "
                      f"on each other); batch time extrapolated linearly in edges"}


def cpu_baseline_forest(K, seconds, n=900, m=9000):
    """The oracle's whole forest-seeded pipeline (forest, closed form, Inc-bSR of the other
    edges) on a smaller graph of the same generator and density, scaled to S entries/s; the
    all-core leg runs independent pipelines side by side."""
    import workloads as W
    s, d = W.chung_lu(n, m, seed=1002)
    path = ORACLE_POOL.stage(n=n, s=s.astype("int64"), d=d.astype("int64"), C=C, K=K)
    return oracle_baseline("forest", path, [0], seconds, float(n) * n, "S entries/s",
                           f"the whole pipeline at n = {n}, m = {m} (same generator and "
                           f"density)")


def cpu_baseline_topk(rows, queries, k, seconds):
    """The oracle's top-k selection on the same stored rows (copied to the host)."""
    import numpy as np
    path = ORACLE_POOL.stage(rows=rows, q=np.asarray(queries), k=k)
    return oracle_baseline("topk", path, list(range(len(queries))), seconds, 1.0, "queries/s",
                           f"selections over {len(queries)} stored rows of the same S")


def cpu_baseline_partitioned(K, parts, p_cross, seconds, n=1200, m=12000):
    """The oracle's whole partitioned pipeline (partition, block fixed points, Inc-bSR of the
    cross edges) on a smaller graph of the same generator and density, scaled to S
    entries/s; the all-core leg runs independent pipelines side by side."""
    import workloads as W
    s, d, _ = W.communities(n, m, parts, p_cross, seed=1102)
    path = ORACLE_POOL.stage(n=n, s=s, d=d, C=C, K=K, parts=parts)
    return oracle_baseline("partitioned", path, [0], seconds, float(n) * n, "S entries/s",
                           f"the whole pipeline at n = {n}, m = {m} ({parts} planted "
                           f"communities, same density)")


def cpu_baseline_gradient(n, s, d, w, a, b, seconds):
    """The oracle's per-edge gradient (no dense matrices; upstream dL/dS = 1 at each pair),
    one edge per task, scaled to edges/s."""
    import numpy as np
    path = ORACLE_POOL.stage(n=n, s=np.asarray(s, np.int64), d=np.asarray(d, np.int64), w=w,
                             a=a, b=b, C=C)
    return oracle_baseline("gradient", path, list(range(len(s))), seconds, 1.0,
                           "edge-gradients/s",
                           "edge-weight gradients by the oracle's per-edge adjoint form")


if __name__ == "__main__":
    main()
