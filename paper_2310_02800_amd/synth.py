"""Seeded synthetic inputs: temporal graphs and motif query streams.

This module only draws inputs. It holds none of the mining arithmetic, so the
GPU path and the CPU oracle can both be fed from it without sharing any code
that decides a result.

Every generator uses ``numpy.random.Generator(PCG64(seed))``. Edge ids are the
positions after a stable sort by ``(t, src, dst)``: the temporal edge list is
chronologically ordered, as the problem definition assumes (Sec. 2.1), except
that equal timestamps are allowed here.

Workloads (the paper's datasets are not available, so these stand in for
them; the sizes follow the evaluation's graph table, Sec. 6, Table 1):

* ``tiny``     n=1,000, m=20,000, Chung-Lu power law (exponent 2.1), times
               uniform in [0, 1e6), float32 log-normal weights.
* ``wiki``     n=1.1M, m=7.8M, Chung-Lu exponent 2.0 with the expected top
               degree near 1e5, bursty per-source Poisson times over 2e8 s
               (shaped like wiki-talk: 1.14M nodes, 7.83M edges, 6.24 years).
* ``skew``     n=10M, m=50M, Zipf degrees (hubs of degree 1e6+), per-source
               1..20 s spacing within a 1e8 s span.

Motif queries (``random_motif``) are motif-order connected: every edge after
the first touches an already used motif node and adds at most one new one.
"""
from __future__ import annotations

import dataclasses
import math
import os
from concurrent.futures import ThreadPoolExecutor
from typing import List, Optional, Sequence, Tuple

import numpy as np

GEN_VERSION = 1

# Predicate operators, shared numbering with the C ABI (documented in the
# public header): weight OP theta.
PRED_GE, PRED_GT, PRED_LE, PRED_LT = 0, 1, 2, 3
NO_GAP = np.iinfo(np.int64).max


@dataclasses.dataclass
class TemporalGraph:
    """A time-sorted temporal edge list (structure of arrays)."""

    n: int
    src: np.ndarray  # int32[m]
    dst: np.ndarray  # int32[m]
    t: np.ndarray    # int64[m], non-decreasing
    w: Optional[np.ndarray] = None  # float32[m]
    name: str = ""
    labels: Optional[np.ndarray] = None  # int32[n], node labels >= 0
    edge_labels: Optional[np.ndarray] = None  # int32[m], edge labels >= 0 (edge id order)

    @property
    def m(self) -> int:
        return int(self.src.shape[0])


@dataclasses.dataclass
class Motif:
    """A motif query: ordered edges over nodes 0..k-1 plus its limits.

    ``gap`` has l-1 entries (``NO_GAP`` = unconstrained); the predicate, when
    ``pred_edge >= 0``, requires ``w[e_pred_edge] OP theta`` in float32.
    ``anti`` lists temporal anti-edges as (a, b, i, window): no graph edge
    phi(a) -> phi(b) may have a time in [t(e_i), t(e_i) + window].
    ``node_labels`` gives each motif node's required vertex label (-1 = any);
    with ``node_label_hi`` the label must lie in [node_labels[v],
    node_label_hi[v]] instead. ``preds`` adds weight predicates (edge, op,
    theta) beyond the one above; all must hold. ``edge_labels`` gives each
    motif edge an inclusive range (lo, hi) its graph edge's label must lie
    in (lo = -1: any).
    """

    edges: List[Tuple[int, int]]
    delta: int
    gap: Optional[List[int]] = None
    pred_edge: int = -1
    pred_op: int = PRED_GE
    pred_theta: float = 0.0
    anti: Optional[List[Tuple[int, int, int, int]]] = None
    node_labels: Optional[List[int]] = None
    node_label_hi: Optional[List[int]] = None
    preds: Optional[List[Tuple[int, int, float]]] = None
    edge_labels: Optional[List[Tuple[int, int]]] = None

    @property
    def l(self) -> int:
        return len(self.edges)

    @property
    def k(self) -> int:
        return 1 + max(max(a, b) for a, b in self.edges)

    def gaps(self) -> List[int]:
        if self.gap is None:
            return [int(NO_GAP)] * max(self.l - 1, 0)
        return [int(g) for g in self.gap]


@dataclasses.dataclass
class Query:
    motif: Motif
    t_lo: int
    t_hi: int
    enumerate: bool = False
    arrival: float = 0.0  # unit-rate arrival time; scale by 1/qps


def _time_order(n, src, dst, t):
    """The permutation that sorts edges by (t, src, dst), stably; the same as
    np.lexsort((dst, src, t)), computed on fewer packed keys when the value
    ranges allow (much faster at tens of millions of edges)."""
    if t.shape[0] == 0:
        return np.zeros(0, np.int64)
    nb = max(1, int(n - 1).bit_length())
    t0 = int(t.min())
    tb = max(1, int(int(t.max()) - t0).bit_length())
    if tb + 2 * nb <= 63:
        key = ((t - t0).astype(np.int64) << (2 * nb)) | (src.astype(np.int64) << nb) | dst.astype(np.int64)
        return np.argsort(key, kind="stable")
    if tb + nb <= 63:
        key = ((t - t0).astype(np.int64) << nb) | src.astype(np.int64)
        return np.lexsort((dst, key))
    return np.lexsort((dst, src, t))


def _finish(n, src, dst, t, w, name) -> TemporalGraph:
    order = _time_order(n, src, dst, t)
    g = TemporalGraph(
        n=int(n),
        src=np.ascontiguousarray(src[order], dtype=np.int32),
        dst=np.ascontiguousarray(dst[order], dtype=np.int32),
        t=np.ascontiguousarray(t[order], dtype=np.int64),
        w=None if w is None else np.ascontiguousarray(w[order], dtype=np.float32),
        name=name,
    )
    return g


def _draw_nodes(rng, cdf, count):
    u = rng.random(count)
    if count < (1 << 22):
        idx = np.searchsorted(cdf, u, side="right")
    else:  # the same lookups, split over threads
        cuts = np.linspace(0, count, 17).astype(np.int64)
        with ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
            parts = list(ex.map(lambda ab: np.searchsorted(cdf, u[ab[0]:ab[1]], side="right"),
                                zip(cuts[:-1], cuts[1:])))
        idx = np.concatenate(parts)
    return np.minimum(idx, cdf.shape[0] - 1).astype(np.int64)


def _chung_lu_pairs(rng, weights, m):
    """Sources and destinations drawn independently in proportion to
    ``weights``; self-loops are redrawn (destination side)."""
    cdf = np.cumsum(weights / weights.sum())
    src = _draw_nodes(rng, cdf, m)
    dst = _draw_nodes(rng, cdf, m)
    bad = np.nonzero(src == dst)[0]
    while bad.size:
        dst[bad] = _draw_nodes(rng, cdf, bad.size)
        bad = bad[src[bad] == dst[bad]]
    return src, dst


def tiny_graph(seed: int = 0, n: int = 1000, m: int = 20000) -> TemporalGraph:
    rng = np.random.Generator(np.random.PCG64(seed))
    wts = (np.arange(n, dtype=np.float64) + 1.0) ** (-1.0 / (2.1 - 1.0))
    src, dst = _chung_lu_pairs(rng, wts, m)
    t = np.sort(rng.integers(0, 1_000_000, m, dtype=np.int64))
    w = rng.lognormal(0.0, 1.0, m).astype(np.float32)
    return _finish(n, src, dst, t, w, f"tiny(n={n},m={m},seed={seed})")


def _wiki_offset(n, m, top):
    """i0 such that m * w_0 / sum(w) == top for w_i = 1/(i+i0)."""
    idx = np.arange(n, dtype=np.float64)

    def top_deg(i0):
        return m * (1.0 / i0) / np.sum(1.0 / (idx + i0))

    lo, hi = 1e-3, 1e7
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        if top_deg(mid) > top:
            lo = mid
        else:
            hi = mid
    return math.sqrt(lo * hi)


def _segment_starts(keys_sorted):
    """Start offsets and lengths of equal-key runs in a sorted key array."""
    if keys_sorted.size == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    brk = np.nonzero(np.diff(keys_sorted))[0] + 1
    starts = np.concatenate(([0], brk)).astype(np.int64)
    lens = np.diff(np.concatenate((starts, [keys_sorted.size]))).astype(np.int64)
    return starts, lens


def _segmented_cumsum(vals, starts, lens):
    cs = np.cumsum(vals)
    base = np.concatenate(([0.0], cs))[starts]
    return cs - np.repeat(base, lens)


def wiki_graph(seed: int = 1, n: int = 1_100_000, m: int = 7_800_000,
               top_degree: float = 1e5, span: float = 2e8) -> TemporalGraph:
    rng = np.random.Generator(np.random.PCG64(seed))
    i0 = _wiki_offset(n, m, top_degree)
    wts = 1.0 / (np.arange(n, dtype=np.float64) + i0)
    src, dst = _chung_lu_pairs(rng, wts, m)
    # bursty per-source Poisson process, log-normal rate, start uniform in span
    order = np.argsort(src, kind="stable")
    s_sorted = src[order]
    starts, lens = _segment_starts(s_sorted)
    nodes = s_sorted[starts]
    z = rng.standard_normal(n)
    start_t = rng.random(n) * span
    rate = (lens.astype(np.float64) / span) * np.exp(2.0 * z[nodes])
    gaps = rng.standard_exponential(m) / np.repeat(rate, lens)
    times = np.repeat(start_t[nodes], lens) + _segmented_cumsum(gaps, starts, lens)
    t_sorted = np.floor(np.mod(times, span)).astype(np.int64)
    t = np.empty(m, np.int64)
    t[order] = t_sorted
    w = rng.lognormal(0.0, 1.0, m).astype(np.float32)
    return _finish(n, src, dst, t, w, f"wiki(n={n},m={m},seed={seed})")


def skew_graph(seed: int = 2, n: int = 10_000_000, m: int = 50_000_000,
               span: int = 100_000_000) -> TemporalGraph:
    rng = np.random.Generator(np.random.PCG64(seed))
    wts = 1.0 / (np.arange(n, dtype=np.float64) + 1.0)
    src, dst = _chung_lu_pairs(rng, wts, m)
    order = np.argsort(src, kind="stable")
    s_sorted = src[order]
    starts, lens = _segment_starts(s_sorted)
    nodes = s_sorted[starts]
    lim = np.maximum(0, span - 20 * lens)
    start_t = rng.integers(0, lim + 1)
    gaps = rng.integers(1, 21, m).astype(np.int64)
    cs = np.cumsum(gaps)
    base = np.concatenate(([0], cs))[starts]
    t_sorted = np.repeat(start_t, lens) + cs - np.repeat(base, lens)
    t = np.empty(m, np.int64)
    t[order] = t_sorted
    del nodes
    return _finish(n, src, dst, t, None, f"skew(n={n},m={m},seed={seed})")


def random_graph(rng: np.random.Generator, n: int, m: int, t_max: int,
                 self_loops: bool = True, weights: bool = True) -> TemporalGraph:
    """Small uniform random graph for exhaustive tests (ties and, optionally,
    self-loops allowed)."""
    src = rng.integers(0, n, m)
    dst = rng.integers(0, n, m)
    if not self_loops:
        bad = src == dst
        dst[bad] = (dst[bad] + 1 + rng.integers(0, n - 1, int(bad.sum()))) % n
    t = rng.integers(0, t_max + 1, m).astype(np.int64)
    w = rng.lognormal(0.0, 1.0, m).astype(np.float32) if weights else None
    return _finish(n, src, dst, t, w, f"random(n={n},m={m})")


# ---------------------------------------------------------------- motifs

def random_motif(rng: np.random.Generator, l: int, k: int) -> List[Tuple[int, int]]:
    """A motif-order connected motif with exactly ``l`` edges and ``k`` nodes.

    Edge 0 is (0, 1); each later edge touches a used node and adds at most one
    new node, numbered in order of first appearance; no edge has a == b.
    """
    if not (2 <= k <= l + 1):
        raise ValueError("need 2 <= k <= l+1")
    news = set(rng.choice(np.arange(1, l), size=k - 2, replace=False).tolist()) if k > 2 else set()
    edges = [(0, 1)]
    used = 2
    for i in range(1, l):
        if i in news:
            x = int(rng.integers(0, used))
            y = used
            used += 1
            edges.append((x, y) if rng.random() < 0.5 else (y, x))
        else:
            x, y = rng.choice(used, size=2, replace=False).tolist()
            edges.append((int(x), int(y)))
    return edges


def _log_uniform_int(rng, lo, hi):
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def batch_queries(seed: int = 3, q: int = 64) -> List[Motif]:
    """64 mixed motifs over the tiny graph: l in 3..6, k in 3..min(5, l+1),
    delta log-uniform in [600, 86400]; odd queries carry a weight predicate."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(q):
        l = int(rng.integers(3, 7))
        k = int(rng.integers(3, min(5, l + 1) + 1))
        edges = random_motif(rng, l, k)
        delta = _log_uniform_int(rng, 600, 86400)
        mot = Motif(edges=edges, delta=delta)
        if i % 2 == 1:
            mot.pred_edge = int(rng.integers(0, l))
            mot.pred_op = PRED_GE if rng.random() < 0.5 else PRED_LT
            mot.pred_theta = float(np.float32(math.exp(rng.standard_normal())))
        out.append(mot)
    return out


def serve_queries(t_min: int, t_max: int, seed: int = 4, q: int = 10_000,
                  enum_frac: float = 0.1, delta_range=(600, 86400)) -> List[Query]:
    """A query stream: motifs as in ``batch_queries`` (delta log-uniform over
    ``delta_range``), a root time range covering 1-100% of the span, 10%
    enumerate requests, unit-rate Poisson arrival times."""
    rng = np.random.Generator(np.random.PCG64(seed))
    span = t_max - t_min
    arrivals = np.cumsum(rng.standard_exponential(q))
    out = []
    for i in range(q):
        l = int(rng.integers(3, 7))
        k = int(rng.integers(3, min(5, l + 1) + 1))
        edges = random_motif(rng, l, k)
        mot = Motif(edges=edges, delta=_log_uniform_int(rng, delta_range[0], delta_range[1]))
        if i % 2 == 1:
            mot.pred_edge = int(rng.integers(0, l))
            mot.pred_op = PRED_GE if rng.random() < 0.5 else PRED_LT
            mot.pred_theta = float(np.float32(math.exp(rng.standard_normal())))
        f = rng.uniform(0.01, 1.0)
        width = int(f * span)
        lo = int(t_min + rng.integers(0, max(span - width, 0) + 1))
        out.append(Query(motif=mot, t_lo=lo, t_hi=lo + width,
                         enumerate=bool(rng.random() < enum_frac),
                         arrival=float(arrivals[i])))
    return out


# Named motifs of the at-scale workloads.
TRIANGLE = [(0, 1), (1, 2), (2, 0)]
FOUR_CYCLE = [(0, 1), (1, 2), (2, 3), (3, 0)]
OUT_STAR3 = [(0, 1), (0, 2), (0, 3)]
SKEW_MOTIF = [(0, 1), (1, 2), (2, 3), (3, 0), (0, 2)]


def wiki_queries() -> List[Motif]:
    """The six count runs on the wiki-shaped graph."""
    out = []
    for d in (3600, 86400):
        for e in (TRIANGLE, FOUR_CYCLE, OUT_STAR3):
            out.append(Motif(edges=list(e), delta=d))
    return out


def skew_query() -> Motif:
    return Motif(edges=list(SKEW_MOTIF), delta=3600, gap=[600, 600, 600, 600])


def tiny_query() -> Motif:
    return Motif(edges=list(TRIANGLE), delta=10_000)


def content_hash(g: TemporalGraph) -> str:
    import hashlib
    h = hashlib.sha256()
    for a in (g.src, g.dst, g.t) + ((g.w,) if g.w is not None else ()):
        h.update(np.ascontiguousarray(a).tobytes())
    if g.labels is not None:
        h.update(b"labels")
        h.update(np.ascontiguousarray(g.labels).tobytes())
    if g.edge_labels is not None:
        h.update(b"edge_labels")
        h.update(np.ascontiguousarray(g.edge_labels).tobytes())
    return h.hexdigest()[:16]


def node_labels(seed: int, n: int, n_labels: int) -> np.ndarray:
    """Uniform random vertex labels 0..n_labels-1 (the paper's labels are
    randomly generated, Sec. 6)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, n_labels, n).astype(np.int32)


def with_labels(g: TemporalGraph, labels) -> TemporalGraph:
    return dataclasses.replace(g, labels=np.ascontiguousarray(labels, dtype=np.int32))


def edge_labels(seed: int, m: int, n_labels: int) -> np.ndarray:
    """Uniform random edge labels 0..n_labels-1 (random edge features, as the
    paper attaches to its non-attributed graphs, Sec. 6)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, n_labels, m).astype(np.int32)


def with_edge_labels(g: TemporalGraph, labels) -> TemporalGraph:
    return dataclasses.replace(g, edge_labels=np.ascontiguousarray(labels, dtype=np.int32))
