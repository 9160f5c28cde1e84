"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module holds graph and update-stream generators only. It contains none of the
SimRank arithmetic: it draws edges, update streams, edge weights, loss pairs and
column samples, and keeps the integer bookkeeping (which edges currently exist)
that a stream generator needs to emit valid insertions and deletions.

The paper's datasets (DBLP, CitH, YouTube, web and social graphs) and its GraphGen
synthetic generator are not available, so directed Chung-Lu power-law graphs stand
in for them:

* node weight ``omega_v = (v + 1) ** (-1 / (exponent - 1))`` (exponent 2.1),
* out-weights and in-weights are ``omega`` under two independent seeded permutations,
* an edge ``(s, t)`` draws ``s`` proportional to the out-weight and ``t`` proportional
  to the in-weight; self-loops and duplicates are rejected until exactly ``m`` distinct
  edges exist (hubs saturate; that is part of the recipe).

Random numbers come from NumPy's PCG64 generator. Seeds follow one rule per workload:
graph ``1000 + c``, update stream ``2000 + c``, pairs and weights ``3000 + c`` for
workload number ``c``.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "WORKLOADS",
    "chung_lu",
    "insertion_stream",
    "mixed_stream",
    "batch_stream",
    "lognormal_weights",
    "loss_pairs",
    "column_sample",
    "with_hubs",
    "existing_batch",
    "existing_batches",
    "communities",
    "rng",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


# The five workloads: sizes and parameters (C damping, K series depth).
WORKLOADS = {
    1: dict(name="c0_unit_fp64_n1k", n=1_000, m=5_000, C=0.6, K=15, updates=20),
    2: dict(name="c0_stream_hilo_n20k", n=20_000, m=200_000, C=0.6, K=15, updates=1_000,
            p_insert=0.7),
    3: dict(name="batch_nodes_n50k", n=50_000, m=1_000_000, C=0.6, K=15, batches=16,
            max_batch=4096),
    4: dict(name="column_sweep_n1m", n=1_000_000, m=10_000_000, C=0.6, K=10, K_ps=30,
            updates=100, columns=65_536, block=8_192),
    5: dict(name="adjoint_weighted_n20k", n=20_000, m=200_000, C=0.6, K=15, pairs=4_096,
            fd_edges=64),
}


def chung_lu(n: int, m: int, exponent: float = 2.1, seed: int = 0):
    """Directed Chung-Lu graph with exactly ``m`` distinct edges and no self-loops.

    Returns ``(src, dst)`` as int32 arrays in generation order (an edge is ``src -> dst``).
    """
    if m > n * (n - 1):
        raise ValueError("too many edges for a simple digraph")
    g = rng(seed)
    omega = (np.arange(n, dtype=np.float64) + 1.0) ** (-1.0 / (exponent - 1.0))
    w_out = omega[g.permutation(n)]
    w_in = omega[g.permutation(n)]
    c_out = np.cumsum(w_out)
    c_out /= c_out[-1]
    c_in = np.cumsum(w_in)
    c_in /= c_in[-1]
    keys = np.empty(0, dtype=np.int64)
    rounds = 0
    while keys.size < m:
        need = m - keys.size
        draw = int(need * 1.25) + 64
        s = np.searchsorted(c_out, g.random(draw), side="right")
        t = np.searchsorted(c_in, g.random(draw), side="right")
        np.minimum(s, n - 1, out=s)
        np.minimum(t, n - 1, out=t)
        ok = s != t
        new = s[ok].astype(np.int64) * n + t[ok].astype(np.int64)
        allk = np.concatenate([keys, new])
        _, first = np.unique(allk, return_index=True)
        first.sort()
        keys = allk[first][:m]
        rounds += 1
        if rounds > 10_000:
            raise RuntimeError("Chung-Lu generator did not reach m distinct edges")
    src = (keys // n).astype(np.int32)
    dst = (keys % n).astype(np.int32)
    return src, dst


class _EdgeSet:
    """Current edge set with O(1) membership, insertion and uniform removal.

    Edges are ``(i, j)`` tuples, so the node count may grow while the set is in use.
    """

    def __init__(self, src, dst):
        self.keys = list(zip(src.tolist(), dst.tolist()))
        self.pos = {k: p for p, k in enumerate(self.keys)}

    def __contains__(self, key):
        return key in self.pos

    def add(self, key):
        self.pos[key] = len(self.keys)
        self.keys.append(key)

    def remove(self, key):
        p = self.pos.pop(key)
        last = self.keys.pop()
        if p < len(self.keys):
            self.keys[p] = last
            self.pos[last] = p

    def pick(self, g):
        return self.keys[int(g.integers(len(self.keys)))]

    def __len__(self):
        return len(self.keys)


def _uniform_non_edge(g, n, es, forbid=()):
    while True:
        i = int(g.integers(n))
        j = int(g.integers(n))
        if i == j or (i, j) in es or (i, j) in forbid:
            continue
        return i, j


def insertion_stream(n, src, dst, count, seed):
    """``count`` insertions of uniform non-edges ``(i, j)`` between existing nodes, i != j.

    Returns int32 arrays ``(i, j)``; each insertion sees the edges inserted before it.
    """
    g = rng(seed)
    es = _EdgeSet(src, dst)
    out_i, out_j = [], []
    for _ in range(count):
        i, j = _uniform_non_edge(g, n, es)
        es.add((i, j))
        out_i.append(i)
        out_j.append(j)
    return np.asarray(out_i, np.int32), np.asarray(out_j, np.int32)


def mixed_stream(n, src, dst, count, p_insert, seed):
    """Insert a uniform non-edge with probability ``p_insert``, else delete a uniform
    existing edge of the current graph. Returns int32 ``(i, j)`` and int8 ``op``
    (+1 insert, -1 delete)."""
    g = rng(seed)
    es = _EdgeSet(src, dst)
    oi, oj, oo = [], [], []
    for _ in range(count):
        if g.random() < p_insert or len(es) == 0:
            i, j = _uniform_non_edge(g, n, es)
            es.add((i, j))
            op = 1
        else:
            i, j = es.pick(g)
            es.remove((i, j))
            op = -1
        oi.append(i)
        oj.append(j)
        oo.append(op)
    return (np.asarray(oi, np.int32), np.asarray(oj, np.int32), np.asarray(oo, np.int8))


def batch_stream(n, src, dst, batches, max_batch, seed, min_batch=1, share_frac=0.25,
                 mix=(0.40, 0.20, 0.10, 0.30), p_delete_c0=1.0 / 3.0, cancel_frac=0.02):
    """Mixed batches of edge updates with new-node endpoints and shared sinks.

    Each batch has a size drawn uniformly from ``min_batch..max_batch``. Edge kinds are
    drawn with probabilities ``mix`` = (new source into an existing sink, existing source
    into a new sink, both new, both existing). An existing-existing edge deletes a uniform
    existing edge with probability ``p_delete_c0``, else inserts a uniform non-edge. About
    ``share_frac`` of the edges are emitted in groups of 2..8 that share one sink (the
    sink's newness consistent with the kind), and about ``cancel_frac`` of each batch is
    insert-then-delete pairs of one fresh edge, which cancel inside the batch.

    New node ids are dense: in each batch they are numbered from the current node count
    upward in order of first appearance in the emitted edge list.

    Returns ``(batches, node_counts)``: a list of ``(i, j, op)`` int32/int32/int8 arrays and
    the node count after each batch.
    """
    g = rng(seed)
    es = _EdgeSet(src, dst)
    cur_n = int(n)
    mix = np.asarray(mix, dtype=np.float64)
    mix = mix / mix.sum()
    out, counts = [], []
    for _ in range(batches):
        size = int(g.integers(min_batch, max_batch + 1))
        n_cancel = int(round(size * cancel_frac / 2))
        units = []          # each unit: list of (i, j, op); new nodes as ('new', tag)
        touched = set()     # existing-existing keys used in this batch
        tag = [0]

        def fresh():
            tag[0] += 1
            return ("new", tag[0])

        # a unit is a group of 2..8 edges (mean 5) with probability p_group, chosen so that
        # about share_frac of the edges sit in groups
        p_group = share_frac / (5.0 * (1.0 - share_frac) + share_frac)
        left = size - 2 * n_cancel
        while left > 0:
            gs = min(int(g.integers(2, 9)) if (left >= 2 and g.random() < p_group) else 1,
                     left)
            kind = int(g.choice(4, p=mix))
            unit = []
            if kind == 0:
                j = int(g.integers(cur_n))
                unit = [(fresh(), j, 1) for _ in range(gs)]
            elif kind == 1:
                j = fresh()
                srcs = set()
                while len(srcs) < gs:
                    srcs.add(int(g.integers(cur_n)))
                unit = [(i, j, 1) for i in sorted(srcs)]
            elif kind == 2:
                j = fresh()
                unit = [(fresh(), j, 1) for _ in range(gs)]
            else:
                sink = int(g.integers(cur_n)) if gs > 1 else None
                for _ in range(gs):
                    if g.random() < p_delete_c0 and len(es) > 0:
                        e = None
                        for _ in range(64):
                            c = es.pick(g)
                            if (sink is None or c[1] == sink) and c not in touched:
                                e = c
                                break
                        if e is None:
                            continue
                        touched.add(e)
                        unit.append((e[0], e[1], -1))
                    else:
                        for _ in range(1000):
                            i = int(g.integers(cur_n))
                            j = sink if sink is not None else int(g.integers(cur_n))
                            if i != j and (i, j) not in es and (i, j) not in touched:
                                touched.add((i, j))
                                unit.append((i, j, 1))
                                break
            if unit:
                units.append(unit)
            left -= gs
        for _ in range(n_cancel):
            i, j = _uniform_non_edge(g, cur_n, es, touched)
            touched.add((i, j))
            units.append([(i, j, 1), (i, j, -1)])
        # emit units in a seeded order; a unit's edges stay in order (cancelling pairs keep
        # the insertion first)
        flat = []
        for u in g.permutation(len(units)).tolist():
            flat.extend(units[u])
        remap = {}
        for (a, b, _op) in flat:
            for x in (a, b):
                if isinstance(x, tuple) and x not in remap:
                    remap[x] = cur_n + len(remap)
        fin = [(remap.get(a, a) if isinstance(a, tuple) else a,
                remap.get(b, b) if isinstance(b, tuple) else b, op) for (a, b, op) in flat]
        for (a, b, op) in fin:
            if op == 1:
                es.add((a, b))
            else:
                es.remove((a, b))
        cur_n += len(remap)
        out.append((np.asarray([e[0] for e in fin], np.int32),
                    np.asarray([e[1] for e in fin], np.int32),
                    np.asarray([e[2] for e in fin], np.int8)))
        counts.append(cur_n)
    return out, counts


def lognormal_weights(m, seed, sigma=0.5):
    """Edge weights ``exp(N(0, sigma^2))`` in edge order, float64."""
    return np.exp(rng(seed).normal(0.0, sigma, size=m))


def loss_pairs(n, npairs, seed, t_max=0.2):
    """Unordered node pairs ``a < b`` without replacement and targets ``U(0, t_max)``."""
    g = rng(seed)
    seen = set()
    a_l, b_l = [], []
    while len(a_l) < npairs:
        a = int(g.integers(n))
        b = int(g.integers(n))
        if a == b:
            continue
        a, b = min(a, b), max(a, b)
        if (a, b) in seen:
            continue
        seen.add((a, b))
        a_l.append(a)
        b_l.append(b)
    t = g.uniform(0.0, t_max, size=npairs)
    return np.asarray(a_l, np.int32), np.asarray(b_l, np.int32), t


def column_sample(n, k, seed, extra=()):
    """``k`` distinct seeded node ids plus ``extra`` ids, sorted, int32."""
    g = rng(seed)
    base = g.choice(n, size=min(k, n), replace=False)
    return np.unique(np.concatenate([base, np.asarray(extra, dtype=np.int64)])).astype(np.int32)


def with_hubs(n, src, dst, hubs, seed):
    """Adds edges so that every hub ``(node, in_degree, out_degree)`` has exactly those
    degrees: the new in-neighbours (out-neighbours) of a hub are drawn uniformly, without
    replacement, from the nodes that are neither hubs nor linked to it yet. Raises
    ``ValueError`` when a hub already has more edges than asked. Returns ``(src, dst)`` int32
    arrays: the input edges, then the added ones in generation order."""
    g = rng(seed)
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    hub_ids = np.asarray(sorted({int(h) for h, _, _ in hubs}), dtype=np.int64)
    add_s, add_d = [], []
    for h, want_in, want_out in hubs:
        for want, into in ((want_in, True), (want_out, False)):
            cur = src[dst == h] if into else dst[src == h]
            extra = np.asarray(add_s if into else add_d, dtype=np.int64)
            other = np.asarray(add_d if into else add_s, dtype=np.int64)
            cur = np.concatenate([cur, extra[other == h]]) if len(extra) else cur
            need = want - len(np.unique(cur))
            if need < 0:
                raise ValueError(f"hub {h} already has more than {want} edges")
            cand = np.setdiff1d(np.arange(n, dtype=np.int64),
                                np.concatenate([cur, hub_ids]))
            pick = g.choice(cand, size=need, replace=False)
            if into:
                add_s.extend(pick.tolist())
                add_d.extend([h] * need)
            else:
                add_s.extend([h] * need)
                add_d.extend(pick.tolist())
    return (np.concatenate([src, np.asarray(add_s, dtype=np.int64)]).astype(np.int32),
            np.concatenate([dst, np.asarray(add_d, dtype=np.int64)]).astype(np.int32))


def existing_batch(n, src, dst, n_ins, n_del, shared, seed):
    """A batch between existing nodes: ``n_ins`` insertions of distinct non-edges (the first
    ``shared`` into one uniformly drawn sink, the rest uniform), then ``n_del`` deletions of
    distinct existing edges. Returns int32 arrays ``(src, dst)`` and int8 ops."""
    return existing_batches(n, src, dst, 1, n_ins, n_del, shared, seed)[0]


def existing_batches(n, src, dst, count, n_ins, n_del, shared, seed):
    """``count`` batches shaped as in ``existing_batch`` (each with its own shared sink) that
    can be applied one after another: no edge appears in two of them, insertions are non-edges
    of the original graph and deletions are distinct original edges. Returns a list of
    ``(src, dst, ops)`` triples."""
    g = rng(seed)
    es = set(zip(np.asarray(src).tolist(), np.asarray(dst).tolist()))
    new = set()
    ins = []
    for _ in range(count):
        bi, bj = [], []
        sink = int(g.integers(n))
        while len(bi) < n_ins:
            a = int(g.integers(n))
            b = sink if len(bi) < shared else int(g.integers(n))
            if a != b and (a, b) not in es and (a, b) not in new:
                new.add((a, b))
                bi.append(a)
                bj.append(b)
        ins.append((bi, bj))
    dels = g.choice(len(src), size=n_del * count, replace=False).tolist()
    out = []
    for t, (bi, bj) in enumerate(ins):
        for e in dels[t * n_del:(t + 1) * n_del]:
            bi.append(int(src[e]))
            bj.append(int(dst[e]))
        ops = [1] * n_ins + [-1] * n_del
        out.append((np.asarray(bi, dtype=np.int32), np.asarray(bj, dtype=np.int32),
                    np.asarray(ops, dtype=np.int8)))
    return out


def communities(n, m, parts, p_cross, seed):
    """A digraph with planted communities: nodes are dealt into ``parts`` groups of near-equal
    size under a seeded permutation (so a group's ids are scattered), each group holds a
    Chung-Lu graph on its own nodes, and a fraction ``p_cross`` of the m edges joins uniformly
    drawn nodes of different groups. Returns int32 ``(src, dst)`` and the int32 group of every
    node (the planted labels, for reference)."""
    g = rng(seed)
    perm = g.permutation(n)
    group = np.empty(n, dtype=np.int32)
    sizes = [n // parts + (1 if p < n % parts else 0) for p in range(parts)]
    members, start = [], 0
    for p, sz in enumerate(sizes):
        members.append(perm[start:start + sz])
        group[perm[start:start + sz]] = p
        start += sz
    n_cross = int(round(m * p_cross)) if parts > 1 else 0
    src, dst = [], []
    left = m - n_cross
    for p, mem in enumerate(members):
        mp = left // (parts - p)
        left -= mp
        s, d = chung_lu(len(mem), mp, seed=int(g.integers(1 << 31)))
        src.append(mem[s])
        dst.append(mem[d])
    es = set(zip(np.concatenate(src).tolist(), np.concatenate(dst).tolist()))
    cs, cd = [], []
    while len(cs) < n_cross:
        a, b = (int(v) for v in g.integers(n, size=2))
        if group[a] != group[b] and (a, b) not in es:
            es.add((a, b))
            cs.append(a)
            cd.append(b)
    src = np.concatenate(src + [np.asarray(cs, dtype=np.int64)]).astype(np.int32)
    dst = np.concatenate(dst + [np.asarray(cd, dtype=np.int64)]).astype(np.int32)
    order = g.permutation(len(src))
    return src[order], dst[order], group
