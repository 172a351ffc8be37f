"""Shared test helpers: graph transforms and closed-form counts.

The closed forms below are written from the problem definition (Sec. 2.1)
for motifs small enough to count without a search; they pin the oracle.
"""
from __future__ import annotations

import itertools
import json
import os

import numpy as np

from paper_2310_02800_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
I64_MAX = np.iinfo(np.int64).max
I64_MIN = np.iinfo(np.int64).min


def graph_from_edges(n, triples, w=None):
    arr = np.array(triples, dtype=np.int64).reshape(-1, 3)
    src, dst, t = arr[:, 0], arr[:, 1], arr[:, 2]
    order = np.lexsort((dst, src, t))
    ww = None if w is None else np.asarray(w, np.float32)[order]
    return synth.TemporalGraph(n=n, src=src[order].astype(np.int32), dst=dst[order].astype(np.int32),
                               t=t[order].astype(np.int64), w=ww)


def resort(n, src, dst, t, w):
    order = np.lexsort((dst, src, t))
    return synth.TemporalGraph(n=n, src=np.ascontiguousarray(src[order], np.int32),
                               dst=np.ascontiguousarray(dst[order], np.int32),
                               t=np.ascontiguousarray(t[order], np.int64),
                               w=None if w is None else np.ascontiguousarray(w[order], np.float32))


def reverse_edges(g):
    return resort(g.n, g.dst.copy(), g.src.copy(), g.t.copy(), None if g.w is None else g.w.copy())


def reverse_time(g):
    T = int(g.t.max()) if g.m else 0
    return resort(g.n, g.src.copy(), g.dst.copy(), (T - g.t).astype(np.int64), None if g.w is None else g.w.copy())


def relabel(g, rng):
    perm = rng.permutation(g.n).astype(np.int64)
    return resort(g.n, perm[g.src], perm[g.dst], g.t.copy(), None if g.w is None else g.w.copy())


def all_connected_motifs(max_l, max_k):
    """Every motif-order connected motif with l <= max_l edges, k <= max_k
    nodes: edge 0 is (0,1); each later edge joins used nodes or one used node
    and the next new node, in either direction."""
    out = []

    def rec(edges, used):
        out.append(list(edges))
        if len(edges) == max_l:
            return
        opts = [(x, y) for x in range(used) for y in range(used) if x != y]
        if used < max_k:
            opts += [(x, used) for x in range(used)] + [(used, x) for x in range(used)]
        for e in opts:
            rec(edges + [e], used + (1 if used in e else 0))

    rec([(0, 1)], 2)
    return out


# ---------------------------------------------------------------- closed forms

def cf_single_edge(g, t_lo=I64_MIN, t_hi=I64_MAX):
    """l = 1: every non-self-loop edge whose time is in the root range."""
    sel = (g.src != g.dst) & (g.t >= t_lo) & (g.t <= t_hi)
    return int(sel.sum())


def cf_repeat_pair(g, delta):
    """Motif a->b, a->b: pairs of edges on the same ordered node pair with
    0 < t_j - t_i <= delta (counted by two pointers per pair)."""
    keep = g.src != g.dst
    s, d, t = g.src[keep].astype(np.int64), g.dst[keep].astype(np.int64), g.t[keep]
    order = np.lexsort((t, d, s))
    s, d, t = s[order], d[order], t[order]
    total = 0
    i = 0
    m = s.size
    while i < m:
        j = i
        while j < m and s[j] == s[i] and d[j] == d[i]:
            j += 1
        ts = t[i:j]
        lo = hi = 0
        for a in range(ts.size):
            while lo < ts.size and ts[lo] <= ts[a]:
                lo += 1
            hi = max(hi, lo)
            while hi < ts.size and ts[hi] <= ts[a] + delta:
                hi += 1
            total += hi - lo
        i = j
    return total


def _out_lists(g):
    order = np.lexsort((g.t, g.src))
    s = g.src[order]
    starts = np.searchsorted(s, np.arange(g.n + 1), side="left")
    return order, starts


def cf_two_path(g, delta):
    """Motif a->b, b->c: for every root (u,v,t) with u != v, the out-edges of
    v with time in (t, t+delta] whose head is neither u nor v."""
    order, starts = _out_lists(g)
    ot = g.t[order]
    od = g.dst[order]
    total = 0
    for r in range(g.m):
        u, v, t = int(g.src[r]), int(g.dst[r]), int(g.t[r])
        if u == v:
            continue
        b, e = starts[v], starts[v + 1]
        lo = b + np.searchsorted(ot[b:e], t, side="right")
        hi = b + np.searchsorted(ot[b:e], t + delta, side="right")
        heads = od[lo:hi]
        total += int(np.sum((heads != u) & (heads != v)))
    return total


def cf_reciprocal(g, delta):
    """Motif a->b, b->a: for every root (u,v,t) with u != v, the edges v->u
    with time in (t, t+delta]."""
    order, starts = _out_lists(g)
    ot = g.t[order]
    od = g.dst[order]
    total = 0
    for r in range(g.m):
        u, v, t = int(g.src[r]), int(g.dst[r]), int(g.t[r])
        if u == v:
            continue
        b, e = starts[v], starts[v + 1]
        lo = b + np.searchsorted(ot[b:e], t, side="right")
        hi = b + np.searchsorted(ot[b:e], t + delta, side="right")
        total += int(np.sum(od[lo:hi] == u))
    return total


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)
