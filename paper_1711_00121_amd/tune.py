"""Autotuner of the fused batch pass (argument marshalling and bookkeeping only; the timing
runs in the library's kernels).

A batch of apply_batch defers its low-rank blocks into a panel and applies every
``batch_chunk`` of them in one fused pass over S (a GEMM on the FP64 matrix cores); each
deferred block also corrects the columns that the chunk's later blocks read. Per block, the
pass costs ``gemm(chunk) / chunk`` and the corrections grow with the chunk. The tuner times
both on the device at the context's size (``sr_time_fused``: a zero panel, so S keeps its
values) for every GEMM tile variant (panel columns per LDS chunk, LDS pitch) and every
candidate chunk, picks the cheapest per block, sets it on the context, and caches the choice
in a JSON file keyed by node-count bucket, K and store precision.
"""
from __future__ import annotations

import json
import os
import tempfile

# tile variants of the fused GEMM: (panel columns per LDS chunk, LDS pitch) on the float64
# matrix cores, and the float32 matrix cores' variant (SR_UPDATE_FP32; pitch in floats)
VARIANTS = {0: (16, 18), 1: (16, 20), 2: (32, 34), 3: (32, 36)}
F32_VARIANT = 4
F32_TILE = (32, 33)
CHUNKS = (32, 48, 64, 96, 128)
BUCKET = 8192


def cache_path():
    base = os.environ.get("SR_TUNE_CACHE")
    if base:
        return base
    root = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    return os.path.join(root, "paper_1711_00121_amd", "fused_tuning.json")


def key_for(n, K, prec):
    return f"n{max(1, round(n / BUCKET)) * BUCKET}_K{K}_{prec}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, data):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=os.path.dirname(os.path.abspath(path)), suffix=".tmp")
    with os.fdopen(fd, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune(ctx, chunks=CHUNKS, variants=None, reps=2, path=None, force=False):
    """Chooses batch_chunk and the GEMM variant for ``ctx`` (a dense-mode Context), applies
    them, and returns a record of the choice (and of the timings when it measured). A context
    whose fused passes run on the float32 matrix cores tunes the chunk of that variant."""
    from . import _lib as L
    path = path or cache_path()
    n, _ = ctx.sizes()
    prec = {L.SR_S_FP64: "fp64", L.SR_S_FP32_HILO: "hilo", L.SR_S_FP32: "fp32"}[ctx.cfg.s_prec]
    f32 = ctx.cfg.update_prec == L.SR_UPDATE_FP32
    if variants is None:
        variants = (F32_VARIANT,) if f32 else tuple(VARIANTS)
    key = key_for(n, ctx.cfg.K, prec) + ("_f32update" if f32 else "")
    data = _load(path)
    if key in data and not force:
        c = data[key]
        ctx.set_tuning(c["batch_chunk"], c["variant"])
        return dict(c, key=key, cached=True)
    table = []
    for v in variants:
        for b in chunks:
            g, c = ctx.time_fused(v, b, reps)
            table.append({"variant": v, "chunk": b, "gemm_ms": round(g, 4),
                          "corr_ms": round(c, 5), "ms_per_block": g / b + c})
    best = min(table, key=lambda t: t["ms_per_block"])
    tile = VARIANTS.get(best["variant"], F32_TILE)
    choice = {"batch_chunk": best["chunk"], "variant": best["variant"],
              "lds_chunk": tile[0], "lds_pitch": tile[1],
              "ms_per_block": best["ms_per_block"], "n_timed": n}
    data = _load(path)
    data[key] = choice
    _store(path, data)
    ctx.set_tuning(choice["batch_chunk"], choice["variant"])
    return dict(choice, key=key, cached=False, table=table)
