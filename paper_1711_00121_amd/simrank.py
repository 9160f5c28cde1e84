"""Python front of libsimrank: argument marshalling only. Every step of the incremental
method runs in the library's HIP kernels; torch provides device memory and the stream."""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L

_PREC = {"fp64": L.SR_S_FP64, "hilo": L.SR_S_FP32_HILO, "fp32": L.SR_S_FP32}
_MODE = {"dense": L.SR_DENSE, "column": L.SR_COLUMN}
_GAMMA = {"closed": L.SR_GAMMA_CLOSED, "direct": L.SR_GAMMA_DIRECT}
_UPDATE = {"fp64": L.SR_UPDATE_FP64, "fp32": L.SR_UPDATE_FP32}


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _ptr(arr, ctype):
    return arr.ctypes.data_as(C.POINTER(ctype))


def _dev(t):
    return C.c_void_p(t.data_ptr())


def default_config(**kw):
    lib = L.load()
    cfg = L.sr_config()
    L.check(lib.sr_default_config(C.byref(cfg)), "sr_default_config")
    for k, v in kw.items():
        if k == "s_prec":
            v = _PREC[v] if isinstance(v, str) else v
        elif k == "mode":
            v = _MODE[v] if isinstance(v, str) else v
        elif k == "gamma_form":
            v = _GAMMA[v] if isinstance(v, str) else v
        elif k == "update_prec":
            v = _UPDATE[v] if isinstance(v, str) else v
        elif k in ("prune", "fused_batch", "profile", "graphs", "block_store", "tile_skip"):
            v = int(bool(v))
        setattr(cfg, k, v)
    return cfg


def device_bytes(reset_peak=False):
    """(held, peak): device bytes the library holds now over all contexts, and the peak since
    the last reset (``reset_peak`` starts a new peak from what is held now)."""
    held, peak = C.c_int64(), C.c_int64()
    L.check(L.load().sr_device_bytes(C.byref(held), C.byref(peak), int(bool(reset_peak))),
            "sr_device_bytes")
    return held.value, peak.value


def partition(n, src, dst, parts):
    """Block labels from the library's breadth-first partitioner (host only)."""
    src = _i32(src)
    dst = _i32(dst)
    out = np.empty(int(n), dtype=np.int32)
    L.check(L.load().sr_partition(int(n), int(len(src)), _ptr(src, C.c_int32),
                                  _ptr(dst, C.c_int32), int(parts), _ptr(out, C.c_int32)),
            "sr_partition")
    return out


class Context:
    """One incremental-SimRank context on the current CUDA (HIP) device and stream.

    ``Context(n, src, dst, weight=None, S0=None, **config)`` builds the graph and the initial
    S (fixed point of eq (03a) on the device unless ``S0`` is given). Config keys follow
    ``sr_config``: C, K, K_ps, s_prec ('fp64' | 'hilo' | 'fp32'), mode ('dense' | 'column'),
    gamma_form ('closed' | 'direct'), prune, node_cap, edge_cap, init_tol, init_max_iter,
    batch_chunk, fused_batch, split_rows, profile, graphs, update_prec ('fp64' | 'fp32'),
    block_store (partitioned contexts: S kept per pair of blocks, Example 1.1), tile_skip
    (fused passes skip the k-steps whose xi factors vanish on a tile; the same S bit for bit).
    """

    def __init__(self, n, src, dst, weight=None, S0=None, stream=None, init="fixed_point",
                 part=None, parts=None, **config):
        """``init="forest"`` seeds S from a breadth-first spanning forest and applies the
        other edges as one batch (Example 1.2); ``init="partitioned"`` computes S of the
        blocks ``part`` (labels per node, or ``parts`` blocks from ``partition``) block by
        block and applies the cross-block edges as one batch (Example 1.1). The batch's
        statistics are kept in ``self.init_stats``."""
        self.lib = L.load()
        self.cfg = default_config(**config)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        src = _i32(src)
        dst = _i32(dst)
        w = None
        if weight is not None:
            w = np.ascontiguousarray(np.asarray(weight, dtype=np.float64))
        s0 = None
        if S0 is not None:
            s0 = S0.to(device="cuda", dtype=torch.float64).contiguous()
        handle = C.c_void_p()
        self.init_stats = None
        if init == "forest":
            if w is not None or s0 is not None:
                raise ValueError("a forest-seeded context is unweighted and computes its own S")
            s = L.sr_batch_stats()
            st = self.lib.init_simrank_tree(
                C.byref(handle), int(n), int(len(src)), _ptr(src, C.c_int32),
                _ptr(dst, C.c_int32), C.byref(self.cfg), C.c_void_p(self.stream.cuda_stream),
                C.byref(s))
            L.check(st, "init_simrank_tree")
            self.init_stats = {f: getattr(s, f) for f, _ in L.sr_batch_stats._fields_}
            self.init_stats["blocks_case"] = list(s.blocks_case)
            self.h = handle
            self.m0 = len(src)
            return
        if init == "partitioned":
            if w is not None or s0 is not None:
                raise ValueError("a partitioned context is unweighted and computes its own S")
            if part is None:
                part = partition(n, src, dst, parts)
            self.part = _i32(part)
            if len(self.part) != n:
                raise ValueError("part needs one label per node")
            s = L.sr_batch_stats()
            st = self.lib.init_simrank_partitioned(
                C.byref(handle), int(n), int(len(src)), _ptr(src, C.c_int32),
                _ptr(dst, C.c_int32), _ptr(self.part, C.c_int32), C.byref(self.cfg),
                C.c_void_p(self.stream.cuda_stream), C.byref(s))
            L.check(st, "init_simrank_partitioned")
            self.init_stats = {f: getattr(s, f) for f, _ in L.sr_batch_stats._fields_}
            self.init_stats["blocks_case"] = list(s.blocks_case)
            self.h = handle
            self.m0 = len(src)
            return
        if init != "fixed_point":
            raise ValueError(f"unknown init {init!r}")
        st = self.lib.init_simrank(
            C.byref(handle), int(n), int(len(src)), _ptr(src, C.c_int32), _ptr(dst, C.c_int32),
            _ptr(w, C.c_double) if w is not None else None, C.byref(self.cfg),
            _dev(s0) if s0 is not None else None, C.c_void_p(self.stream.cuda_stream))
        L.check(st, "init_simrank")
        self.h = handle
        self.m0 = len(src)
        self.weights = w

    # ------------------------------------------------------------------ updates
    def apply_edge_update(self, i, j, op=1, stats=False):
        s = L.sr_update_stats() if stats else None
        st = self.lib.apply_edge_update(self.h, int(i), int(j), int(op),
                                        C.byref(s) if s is not None else None)
        L.check(st, "apply_edge_update")
        if s is None:
            return None
        return {f: getattr(s, f) for f, _ in L.sr_update_stats._fields_}

    def apply_weight_update(self, i, j, w, stats=False):
        """Weighted graphs: sets the weight of edge i -> j to w (0 deletes, a missing edge
        is inserted)."""
        s = L.sr_update_stats() if stats else None
        st = self.lib.apply_weight_update(self.h, int(i), int(j), float(w),
                                          C.byref(s) if s is not None else None)
        L.check(st, "apply_weight_update")
        if s is None:
            return None
        return {f: getattr(s, f) for f, _ in L.sr_update_stats._fields_}

    def apply_batch(self, src, dst, op, stats=False):
        src = _i32(src)
        dst = _i32(dst)
        op = np.ascontiguousarray(np.asarray(op, dtype=np.int8))
        s = L.sr_batch_stats() if stats else None
        st = self.lib.apply_batch(self.h, int(len(src)), _ptr(src, C.c_int32),
                                  _ptr(dst, C.c_int32), _ptr(op, C.c_int8),
                                  C.byref(s) if s is not None else None)
        L.check(st, "apply_batch")
        if s is None:
            return None
        out = {f: getattr(s, f) for f, _ in L.sr_batch_stats._fields_}
        out["blocks_case"] = list(s.blocks_case)
        return out

    def apply_batch_columns(self, src, dst, op, cols, out=None, stats=False):
        """Column mode: applies a batch between existing nodes and returns the float64 Delta S
        columns of the whole batch as rows, ``out[t, :] = Delta S[:, cols[t]]``."""
        n, _ = self.sizes()
        src = _i32(src)
        dst = _i32(dst)
        cols = _i32(cols)
        op = np.ascontiguousarray(np.asarray(op, dtype=np.int8))
        if out is None:
            out = torch.empty((len(cols), n), dtype=torch.float64, device="cuda")
        s = L.sr_batch_stats() if stats else None
        st = self.lib.apply_batch_columns(self.h, int(len(src)), _ptr(src, C.c_int32),
                                          _ptr(dst, C.c_int32), _ptr(op, C.c_int8),
                                          _ptr(cols, C.c_int32), int(len(cols)), _dev(out),
                                          out.stride(0), C.byref(s) if s is not None else None)
        L.check(st, "apply_batch_columns")
        if s is None:
            return out
        info = {f: getattr(s, f) for f, _ in L.sr_batch_stats._fields_}
        info["blocks_case"] = list(s.blocks_case)
        return out, info

    # ------------------------------------------------------------------ queries
    def sizes(self):
        n = C.c_int64()
        m = C.c_int64()
        L.check(self.lib.sr_sizes(self.h, C.byref(n), C.byref(m)), "sr_sizes")
        return n.value, m.value

    def edges(self):
        """The current edges ``(src, dst, w)`` in the order backward reports dL/dw."""
        m = C.c_int64()
        L.check(self.lib.sr_edges(self.h, None, None, None, 0, C.byref(m)), "sr_edges")
        src = np.empty(m.value, dtype=np.int32)
        dst = np.empty(m.value, dtype=np.int32)
        w = np.empty(m.value, dtype=np.float64)
        L.check(self.lib.sr_edges(self.h, _ptr(src, C.c_int32), _ptr(dst, C.c_int32),
                                  _ptr(w, C.c_double), m.value, C.byref(m)), "sr_edges")
        return src, dst, w

    def query_column(self, x, what="S"):
        n, _ = self.sizes()
        out = torch.empty(n, dtype=torch.float64, device="cuda")
        w = L.SR_COL_S if what == "S" else L.SR_COL_DELTA
        L.check(self.lib.query_column(self.h, int(x), w, _dev(out)), "query_column")
        return out

    def query_columns(self, cols, out=None):
        """Float32 columns as rows of the result: ``out[t, :] = column cols[t]``."""
        n, _ = self.sizes()
        cols = _i32(cols)
        if out is None:
            out = torch.empty((len(cols), n), dtype=torch.float32, device="cuda")
        L.check(self.lib.query_columns(self.h, _ptr(cols, C.c_int32), len(cols), _dev(out),
                                       out.stride(0)), "query_columns")
        return out

    def query_topk(self, q, k, exclude_self=True, out=None):
        """Top-k most similar nodes of each query, best first (ties to the smaller id):
        returns ``(idx, val)``, int32 and float64 tensors of shape ``(len(q), k)``."""
        q = _i32(q)
        if out is None:
            out = (torch.empty((len(q), k), dtype=torch.int32, device="cuda"),
                   torch.empty((len(q), k), dtype=torch.float64, device="cuda"))
        idx, val = out
        L.check(self.lib.query_topk(self.h, _ptr(q, C.c_int32), len(q), int(k),
                                    int(bool(exclude_self)), _dev(idx), _dev(val)),
                "query_topk")
        return idx, val

    def gather_pairs(self, a, b):
        a = torch.as_tensor(a, dtype=torch.int32, device="cuda").contiguous()
        b = torch.as_tensor(b, dtype=torch.int32, device="cuda").contiguous()
        out = torch.empty(a.numel(), dtype=torch.float64, device="cuda")
        L.check(self.lib.sr_gather_pairs(self.h, a.numel(), _dev(a), _dev(b), _dev(out)),
                "sr_gather_pairs")
        return out

    def S(self):
        n, _ = self.sizes()
        out = torch.empty((n, n), dtype=torch.float64, device="cuda")
        L.check(self.lib.sr_copy_S(self.h, _dev(out), n), "sr_copy_S")
        return out

    def get_aff(self, level=-1):
        n, _ = self.sizes()
        A = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
        B = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
        nA = C.c_int64()
        nB = C.c_int64()
        L.check(self.lib.sr_get_aff(self.h, int(level), _dev(A), C.byref(nA), _dev(B),
                                    C.byref(nB)), "sr_get_aff")
        return A[:nA.value].clone(), B[:nB.value].clone()

    def last_plan(self):
        ln = C.c_int64()
        L.check(self.lib.sr_last_plan(self.h, None, 0, C.byref(ln)), "sr_last_plan")
        buf = np.zeros(max(ln.value, 1), dtype=np.int32)
        L.check(self.lib.sr_last_plan(self.h, _ptr(buf, C.c_int32), ln.value, C.byref(ln)),
                "sr_last_plan")
        flat = buf[:ln.value].tolist()
        plan, p = [], 0
        while p < len(flat):
            case, op, j, dj, delta = flat[p:p + 5]
            plan.append(dict(case=case, op=op, j=j, dj=dj, I=flat[p + 5:p + 5 + delta]))
            p += 5 + delta
        return plan

    def backward(self, a, b, g):
        a = torch.as_tensor(a, dtype=torch.int32, device="cuda").contiguous()
        b = torch.as_tensor(b, dtype=torch.int32, device="cuda").contiguous()
        g = torch.as_tensor(g, dtype=torch.float64, device="cuda").contiguous()
        dw = torch.empty(self.sizes()[1], dtype=torch.float64, device="cuda")
        L.check(self.lib.backward(self.h, a.numel(), _dev(a), _dev(b), _dev(g), _dev(dw)),
                "backward")
        return dw

    def time_fused(self, variant, blocks, reps=2):
        """Milliseconds of one fused pass over ``blocks`` deferred blocks with GEMM variant
        ``variant`` at the current size, and of one block's corrections (sr_time_fused)."""
        g = C.c_double()
        c = C.c_double()
        L.check(self.lib.sr_time_fused(self.h, int(variant), int(blocks), int(reps), C.byref(g),
                                       C.byref(c)), "sr_time_fused")
        return g.value, c.value

    def store_bytes(self):
        """(bytes, pairs): bytes of the store of S, and the block pairs held (block store)."""
        b, np_ = C.c_int64(), C.c_int64()
        L.check(self.lib.sr_store_bytes(self.h, C.byref(b), C.byref(np_)), "sr_store_bytes")
        return b.value, np_.value

    def config(self):
        """The configuration as resolved at init (capacities, batch_chunk filled in) and as
        changed since by ``set_tuning``: an ``sr_config``."""
        out = L.sr_config()
        L.check(self.lib.sr_get_config(self.h, C.byref(out)), "sr_get_config")
        return out

    def set_tuning(self, batch_chunk, variant):
        L.check(self.lib.sr_set_tuning(self.h, int(batch_chunk), int(variant)), "sr_set_tuning")
        self.cfg.batch_chunk = int(batch_chunk)

    def tune(self, **kw):
        """Autotunes the fused batch pass (see paper_1711_00121_amd.tune)."""
        from .tune import tune
        return tune(self, **kw)

    def profile(self, enable=True):
        L.check(self.lib.sr_profile(self.h, int(bool(enable))), "sr_profile")

    def profile_read(self, reset=True):
        ms = C.c_double()
        cnt = C.c_int64()
        L.check(self.lib.sr_profile_read(self.h, C.byref(ms), C.byref(cnt), int(bool(reset))),
                "sr_profile_read")
        return ms.value, cnt.value

    def synchronize(self):
        L.check(self.lib.sr_synchronize(self.h), "sr_synchronize")

    def close(self):
        if getattr(self, "h", None):
            self.lib.sr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SimRankPairs(torch.autograd.Function):
    """``S[a, b]`` for the context's graph as a function of its edge weights.

    ``forward(weights, context, a, b)`` returns the pair values; ``weights`` must equal the
    context's current (m,) weights in the order of ``Context.edges`` (those it was built
    with until its first update; all ones for an unweighted context), else ValueError. ``backward`` calls the library's adjoint and
    returns dL/dweights.
    """

    @staticmethod
    def forward(ctx, weights, context, a, b):
        # the context holds S of its current weights (those it was built with, or as updates
        # left them, in the order of Context.edges): any other weights would get stale values
        # and gradients, so they are refused
        ref = context.edges()[2] if hasattr(context, "edges") else getattr(context, "weights",
                                                                            None)
        if ref is None:
            ref = np.ones(context.m0)
        w = weights.detach().to(device="cpu", dtype=torch.float64).numpy()
        if w.shape != ref.shape or not np.array_equal(w, ref):
            raise ValueError("weights differ from those the context was built with; build a "
                             "new Context for new weights")
        a = torch.as_tensor(a, dtype=torch.int32, device="cuda").contiguous()
        b = torch.as_tensor(b, dtype=torch.int32, device="cuda").contiguous()
        ctx.context = context
        ctx.save_for_backward(a, b)
        return context.gather_pairs(a, b)

    @staticmethod
    def backward(ctx, grad_out):
        a, b = ctx.saved_tensors
        dw = ctx.context.backward(a, b, grad_out.detach().to(torch.float64).contiguous())
        return dw, None, None, None


def simrank_pairs(weights, context, a, b):
    return SimRankPairs.apply(weights, context, a, b)


def mfma_layout_probe(a, b):
    lib = L.load()
    a = a.to(device="cuda", dtype=torch.float64).contiguous()
    b = b.to(device="cuda", dtype=torch.float64).contiguous()
    out = torch.empty(256, dtype=torch.float64, device="cuda")
    L.check(lib.sr_mfma_layout_probe(_dev(a), _dev(b), _dev(out),
                                     C.c_void_p(torch.cuda.current_stream().cuda_stream)),
            "sr_mfma_layout_probe")
    return out
