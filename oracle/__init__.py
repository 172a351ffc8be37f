"""CPU oracle for exact temporal motif mining — TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package. The product path never imports it and shares no code with it.

Two independent implementations of the problem definition (Sec. 2.1):

* ``count`` / ``enumerate`` call the plain C depth-first search in
  ``tm_oracle.c`` (Algorithm 1 with the fine-grained gap, edge-attribute
  predicate, vertex and edge label, temporal anti-edge and root-range
  constraints of Sec. 2.1 and Sec. 5.4);
* ``brute.py`` checks every ordered l-tuple of distinct edges against the
  definition literally, for tiny graphs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tm_oracle.c")
_LIB = os.path.join(_HERE, "libtm_oracle.so")
_lib = None

I64_MAX = np.iinfo(np.int64).max
I64_MIN = np.iinfo(np.int64).min


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (no fast-math: the predicate is an exact
    float32 comparison)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-fPIC", "-shared", "-pthread",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32 = ctypes.c_int64, ctypes.c_int
        lib.oracle_graph_new.restype = P
        lib.oracle_graph_new.argtypes = [i64, i64, P, P, P, P]
        lib.oracle_graph_free.argtypes = [P]
        lib.oracle_count.restype = i32
        lib.oracle_count.argtypes = [P, i32, i32, P, i64, P, i32, i32, ctypes.c_float, i64, i64, i32,
                                     i32, P, P, P, i32, P, P, P, P, P, i32, P, P]
        lib.oracle_enumerate.restype = i32
        lib.oracle_enumerate.argtypes = [P, i32, i32, P, i64, P, i32, i32, ctypes.c_float, i64, i64,
                                         i32, P, P, P, i32, P, P, P, P, P, P, ctypes.c_uint64, P]
        lib.oracle_graph_set_labels.argtypes = [P, P]
        lib.oracle_graph_set_edge_labels.argtypes = [P, P]
        lib.oracle_version.restype = i32
        if lib.oracle_version() != 4:
            raise RuntimeError("stale oracle library: rebuild it with oracle.build()")
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class OracleGraph:
    """Holds the time-sorted edge arrays and the per-node in/out id lists."""

    def __init__(self, n: int, src, dst, t, w=None, labels=None, edge_labels=None):
        lib = _load()
        self.src = np.ascontiguousarray(src, dtype=np.int32)
        self.dst = np.ascontiguousarray(dst, dtype=np.int32)
        self.t = np.ascontiguousarray(t, dtype=np.int64)
        self.w = None if w is None else np.ascontiguousarray(w, dtype=np.float32)
        if self.t.size > 1 and np.any(np.diff(self.t) < 0):
            raise ValueError("oracle expects a time-sorted edge list")
        self.n = int(n)
        self.m = int(self.src.size)
        self._h = lib.oracle_graph_new(self.n, self.m, _ptr(self.src), _ptr(self.dst), _ptr(self.t),
                                       _ptr(self.w))
        self.labels = None
        if labels is not None:
            self.labels = np.ascontiguousarray(labels, dtype=np.int32)
            if self.labels.shape != (self.n,) or (self.n and self.labels.min() < 0):
                raise ValueError("labels: one non-negative int32 per node")
            lib.oracle_graph_set_labels(self._h, _ptr(self.labels))
        self.edge_labels = None
        if edge_labels is not None:
            self.edge_labels = np.ascontiguousarray(edge_labels, dtype=np.int32)
            if self.edge_labels.shape != (self.m,) or (self.m and self.edge_labels.min() < 0):
                raise ValueError("edge_labels: one non-negative int32 per edge")
            lib.oracle_graph_set_edge_labels(self._h, _ptr(self.edge_labels))

    @classmethod
    def from_graph(cls, g) -> "OracleGraph":
        return cls(g.n, g.src, g.dst, g.t, g.w, getattr(g, "labels", None), getattr(g, "edge_labels", None))

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.oracle_graph_free(self._h)
            self._h = None


def _motif_args(motif):
    edges = np.ascontiguousarray(np.array(motif.edges, dtype=np.int32).reshape(-1))
    gaps = np.ascontiguousarray(np.array(motif.gaps(), dtype=np.int64)) if motif.l > 1 else None
    return edges, gaps


def _anti_args(motif):
    """Temporal anti-edges as (a, b, attach edge) triples and their windows."""
    anti = getattr(motif, "anti", None) or []
    if not anti:
        return 0, None, None
    trip = np.ascontiguousarray(np.array([x[:3] for x in anti], dtype=np.int32).reshape(-1))
    win = np.ascontiguousarray(np.array([x[3] for x in anti], dtype=np.int64))
    return len(anti), trip, win


def _label_args(motif):
    """Required label per motif node (-1 = any), or None."""
    lab = getattr(motif, "node_labels", None)
    return None if lab is None else np.ascontiguousarray(np.array(lab, dtype=np.int32))


def _attr_args(motif):
    """Extra weight predicates (count, edges, operators, thresholds), upper
    ends of node label ranges, and edge label ranges (lo, hi per edge)."""
    preds = getattr(motif, "preds", None) or []
    pe = np.ascontiguousarray(np.array([p[0] for p in preds], dtype=np.int32)) if preds else None
    po = np.ascontiguousarray(np.array([p[1] for p in preds], dtype=np.int32)) if preds else None
    pt = np.ascontiguousarray(np.array([p[2] for p in preds], dtype=np.float32)) if preds else None
    hi = getattr(motif, "node_label_hi", None)
    hi = None if hi is None else np.ascontiguousarray(np.array(hi, dtype=np.int32))
    el = getattr(motif, "edge_labels", None)
    el = None if el is None else np.ascontiguousarray(np.array(el, dtype=np.int32).reshape(-1))
    return len(preds), pe, po, pt, hi, el


def count(og: OracleGraph, motif, t_lo: int = I64_MIN, t_hi: int = I64_MAX, nthreads: int = 1,
          list_rule: int = 0, with_stats: bool = False):
    """Number of instances. With ``with_stats`` also returns a dict of the
    work counters (roots, windows, probes, visits, pred_visits, matches)."""
    lib = _load()
    edges, gaps = _motif_args(motif)
    na, trip, win = _anti_args(motif)
    lab = _label_args(motif)
    npd, pe, po, pt, lhi, el = _attr_args(motif)
    out = np.zeros(1, np.uint64)
    st = np.zeros(6, np.uint64)
    rc = lib.oracle_count(og._h, motif.l, motif.k, _ptr(edges), int(motif.delta), _ptr(gaps),
                          int(motif.pred_edge), int(motif.pred_op), float(motif.pred_theta),
                          int(t_lo), int(t_hi), int(list_rule), na, _ptr(trip), _ptr(win), _ptr(lab),
                          npd, _ptr(pe), _ptr(po), _ptr(pt), _ptr(lhi), _ptr(el), int(nthreads),
                          _ptr(out), _ptr(st))
    if rc != 0:
        raise ValueError("oracle rejected the query")
    if with_stats:
        keys = ("roots", "windows", "probes", "visits", "pred_visits", "matches")
        return int(out[0]), {k: int(v) for k, v in zip(keys, st)}
    return int(out[0])


def enumerate(og: OracleGraph, motif, t_lo: int = I64_MIN, t_hi: int = I64_MAX,
              capacity: Optional[int] = None) -> np.ndarray:
    """All instances as an int64[count, l] array (root order, then DFS order)."""
    lib = _load()
    edges, gaps = _motif_args(motif)
    na, trip, win = _anti_args(motif)
    lab = _label_args(motif)
    npd, pe, po, pt, lhi, el = _attr_args(motif)
    n_out = np.zeros(1, np.uint64)
    if capacity is None:
        capacity = count(og, motif, t_lo, t_hi)
    buf = np.zeros((max(capacity, 1), motif.l), np.int64)
    rc = lib.oracle_enumerate(og._h, motif.l, motif.k, _ptr(edges), int(motif.delta), _ptr(gaps),
                              int(motif.pred_edge), int(motif.pred_op), float(motif.pred_theta),
                              int(t_lo), int(t_hi), na, _ptr(trip), _ptr(win), _ptr(lab),
                              npd, _ptr(pe), _ptr(po), _ptr(pt), _ptr(lhi), _ptr(el), _ptr(buf), int(capacity),
                              _ptr(n_out))
    if rc != 0:
        raise ValueError("oracle rejected the query")
    n = int(n_out[0])
    if n > capacity:
        raise ValueError(f"capacity {capacity} < {n} instances")
    return buf[:n].copy()
