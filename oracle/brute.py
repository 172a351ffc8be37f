"""Literal brute force over all ordered l-tuples of distinct edges.

TEST INFRASTRUCTURE ONLY. For tiny graphs (m up to a few dozen) this checks
each condition of the problem definition (Sec. 2.1) directly: strictly
increasing times, the delta window (inclusive), the fine-grained gaps delta_i,
the existence of an injective node map phi with phi(a_i)=src(e_i) and
phi(b_i)=dst(e_i) (isomorphism: a bijection onto the matched nodes),
edge-weight predicates, vertex and edge labels (single values or ranges),
temporal anti-edges (absence of an edge between two
mapped nodes in a closed time range after the attached edge), and the
root-range filter. It shares nothing with the
C oracle or the GPU path.
"""
from __future__ import annotations

import itertools
from typing import List, Tuple

import numpy as np

I64_MAX = np.iinfo(np.int64).max
I64_MIN = np.iinfo(np.int64).min


def _pred(op: int, w: np.float32, theta: np.float32) -> bool:
    if op == 0:
        return bool(w >= theta)
    if op == 1:
        return bool(w > theta)
    if op == 2:
        return bool(w <= theta)
    return bool(w < theta)


def is_instance(g, motif, tup, t_lo=I64_MIN, t_hi=I64_MAX) -> bool:
    l = motif.l
    if len(tup) != l:
        return False
    ts = [int(g.t[e]) for e in tup]
    if not (t_lo <= ts[0] <= t_hi):
        return False
    for i in range(l - 1):
        if not ts[i] < ts[i + 1]:
            return False
    if ts[-1] - ts[0] > motif.delta:
        return False
    gaps = motif.gaps()
    for i in range(l - 1):
        if ts[i + 1] - ts[i] > gaps[i]:
            return False
    phi = {}
    for (a, b), e in zip(motif.edges, tup):
        for mnode, gnode in ((a, int(g.src[e])), (b, int(g.dst[e]))):
            if mnode in phi and phi[mnode] != gnode:
                return False
            phi[mnode] = gnode
    if len(set(phi.values())) != len(phi):  # injective
        return False
    # vertex labels: a motif node with a required label (or label range)
    # maps to a node whose label is that one (lies in the range)
    his = getattr(motif, "node_label_hi", None)
    for v, want in enumerate(getattr(motif, "node_labels", None) or []):
        if want < 0:
            continue
        top = want if his is None else his[v]
        if not want <= int(g.labels[phi[v]]) <= top:
            return False
    # edge labels: each constrained motif edge's graph edge carries a label in range
    for i, (lo, hi) in enumerate(getattr(motif, "edge_labels", None) or []):
        if lo >= 0 and not lo <= int(g.edge_labels[tup[i]]) <= hi:
            return False
    # weight predicates: the single one and any further ones
    preds = ([(motif.pred_edge, motif.pred_op, motif.pred_theta)] if motif.pred_edge >= 0 else [])
    preds += list(getattr(motif, "preds", None) or [])
    for j, op, theta in preds:
        if not _pred(op, np.float32(g.w[tup[j]]), np.float32(theta)):
            return False
    # temporal anti-edges: no graph edge at all (the tuple's own included) from
    # phi(a) to phi(b) with a time in [t(e_i), t(e_i) + window]
    for a, b, i, win in getattr(motif, "anti", None) or []:
        t0 = ts[i]
        for f in range(g.m):
            if int(g.src[f]) == phi[a] and int(g.dst[f]) == phi[b] and t0 <= int(g.t[f]) <= t0 + win:
                return False
    return True


def enumerate_all(g, motif, t_lo=I64_MIN, t_hi=I64_MAX) -> List[Tuple[int, ...]]:
    """Sorted list of every instance (ordered tuples of distinct edge ids)."""
    out = []
    for tup in itertools.permutations(range(g.m), motif.l):
        if is_instance(g, motif, tup, t_lo, t_hi):
            out.append(tuple(tup))
    out.sort()
    return out


def count_all(g, motif, t_lo=I64_MIN, t_hi=I64_MAX) -> int:
    return len(enumerate_all(g, motif, t_lo, t_hi))
