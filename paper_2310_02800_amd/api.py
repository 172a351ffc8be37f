"""Python binding of the C ABI (argument marshalling only).

Every step of the mining runs in the native HIP library; PyTorch is used only
for device buffers (enumeration output) and stream handles.
"""
from __future__ import annotations

import ctypes
import os
import weakref
from typing import Optional, Sequence

import numpy as np

from . import _native as N

I64_MAX = np.iinfo(np.int64).max
I64_MIN = np.iinfo(np.int64).min


def _ptr(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _stream_handle(stream):
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        except ImportError:
            pass
        return None
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _range(t_lo, t_hi):
    if t_lo is None and t_hi is None:
        return None
    r = N.RootRange(I64_MIN if t_lo is None else int(t_lo), I64_MAX if t_hi is None else int(t_hi))
    return r


def _np(a, dtype):
    if a is None:
        return None
    if hasattr(a, "detach"):
        a = a.detach().cpu().numpy()
    return np.ascontiguousarray(a, dtype=dtype)


class Graph:
    def __init__(self, ctx: "Context", handle):
        self._ctx = ctx
        self._h = handle

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        inf = N.GraphInfo()
        N.check(N.lib().tm_graph_get_info(self._h, ctypes.byref(inf)))
        return {f: getattr(inf, f) for f, _ in N.GraphInfo._fields_}

    def set_node_labels(self, labels) -> None:
        """Attach vertex labels (int32 >= 0, one per node)."""
        lab = _np(labels, np.int32)
        if lab.shape != (self.info()["n_nodes"],):
            raise ValueError("one label per node")
        N.check(N.lib().tm_graph_set_node_labels(self._h, _ptr(lab)))

    def set_edge_labels(self, labels) -> None:
        """Attach edge labels (int32 >= 0, one per edge, in the input order
        given to load_graph)."""
        lab = _np(labels, np.int32)
        if lab.shape != (self.info()["n_edges"],):
            raise ValueError("one label per edge")
        N.check(N.lib().tm_graph_set_edge_labels(self._h, _ptr(lab)))

    def edge_order(self) -> np.ndarray:
        m = self.info()["n_edges"]
        out = np.zeros(m, np.int64)
        N.check(N.lib().tm_graph_edge_order(self._h, _ptr(out)))
        return out

    def csr(self, direction: int):
        """(off, nbr, eid, t_rel) of the out- (0) or in- (1) adjacency, sorted
        by time; 2 and 3: the same lists sorted by (neighbour, time)."""
        inf = self.info()
        n, m = inf["n_nodes"], inf["n_edges"]
        off = np.zeros(n + 1, np.uint32)
        nbr = np.zeros(max(m, 1), np.int32)
        eid = np.zeros(max(m, 1), np.int32)
        t = np.zeros(max(m, 1), np.int64)
        N.check(N.lib().tm_graph_copy_csr(self._h, int(direction), _ptr(off), _ptr(nbr), _ptr(eid), _ptr(t)))
        return off, nbr[:m], eid[:m], t[:m]

    def close(self):
        if self._h:
            N.lib().tm_free_graph(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Motif:
    def __init__(self, ctx: "Context", handle, l: int):
        self._ctx = ctx
        self._h = handle
        self.l = l

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            N.lib().tm_free_motif(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_desc(edges, delta, gap=None, pred_edge=-1, pred_op=0, pred_theta=0.0, n_nodes=None, anti=None,
              node_labels=None, node_label_hi=None, preds=None, edge_labels=None):
    """Motif descriptor. ``anti``: temporal anti-edges as (a, b, attach edge,
    window) tuples; ``node_labels``: required vertex label per motif node
    (-1 = any), with ``node_label_hi`` the upper ends of label ranges;
    ``preds``: further weight predicates as (edge, op, theta); ``edge_labels``:
    a (lo, hi) label range per motif edge (lo = -1: any)."""
    e = np.ascontiguousarray(np.array(edges, dtype=np.int32).reshape(-1))
    l = e.size // 2
    k = int(n_nodes) if n_nodes is not None else (int(e.max()) + 1 if e.size else 0)
    g = None if gap is None else np.ascontiguousarray(np.array(gap, dtype=np.int64))
    na = 0 if not anti else len(anti)
    an = ad = None
    if na:
        an = np.ascontiguousarray(np.array([x[:3] for x in anti], dtype=np.int32).reshape(-1))
        ad = np.ascontiguousarray(np.array([x[3] for x in anti], dtype=np.int64))
    nl = None
    if node_labels is not None:
        nl = np.ascontiguousarray(np.array(node_labels, dtype=np.int32))
        if nl.shape != (k,):
            raise ValueError("one label (or -1) per motif node")
    nh = None
    if node_label_hi is not None:
        nh = np.ascontiguousarray(np.array(node_label_hi, dtype=np.int32))
        if nh.shape != (k,):
            raise ValueError("one upper label (or -1) per motif node")
    np_ = 0 if not preds else len(preds)
    pa = None
    if np_:
        pa = (N.EdgePred * np_)(*[N.EdgePred(int(x[0]), int(x[1]), float(x[2])) for x in preds])
    el = None
    if edge_labels is not None:
        el = np.ascontiguousarray(np.array(edge_labels, dtype=np.int32).reshape(-1))
        if el.shape != (2 * l,):
            raise ValueError("one (lo, hi) label range per motif edge")
    ptr = lambda a: None if a is None else ctypes.c_void_p(a.ctypes.data)
    d = N.MotifDesc(k, l, ctypes.c_void_p(e.ctypes.data), int(delta), ptr(g), int(pred_edge), int(pred_op),
                    float(pred_theta), na, ptr(an), ptr(ad), ptr(nl), np_,
                    None if pa is None else ctypes.cast(pa, ctypes.c_void_p), ptr(nh), ptr(el))
    return d, (e, g, an, ad, nl, nh, pa, el)  # keep arrays alive with the descriptor


def motif_desc_of(m):
    """Descriptor of a synth.Motif-like object."""
    return make_desc(m.edges, m.delta, None if m.gap is None else m.gaps(), m.pred_edge, m.pred_op, m.pred_theta,
                     anti=getattr(m, "anti", None), node_labels=getattr(m, "node_labels", None),
                     node_label_hi=getattr(m, "node_label_hi", None), preds=getattr(m, "preds", None),
                     edge_labels=getattr(m, "edge_labels", None))


def motif_source(edges, delta=0, key_bytes=4, **kw) -> str:
    d, keep = make_desc(edges, delta, **kw)
    n = ctypes.c_int64(0)
    N.check(N.lib().tm_motif_source(ctypes.byref(d), key_bytes, None, 0, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value + 1)
    N.check(N.lib().tm_motif_source(ctypes.byref(d), key_bytes, buf, n.value + 1, ctypes.byref(n)))
    return buf.value.decode()


def motif_compile_check(edges, delta=0, key_bytes=4, **kw) -> int:
    d, keep = make_desc(edges, delta, **kw)
    n = ctypes.c_int64(0)
    N.check(N.lib().tm_motif_compile_check(ctypes.byref(d), 1, key_bytes, ctypes.byref(n)))
    return n.value


def generic_compile_check(l: int, key_bytes=4) -> int:
    """Compile the table-driven (tier 1) modules for motifs of ``l`` edges, or
    with ``l`` = 0 their batched module for 1-8 edges (no device)."""
    n = ctypes.c_int64(0)
    N.check(N.lib().tm_generic_compile_check(int(l), key_bytes, ctypes.byref(n)))
    return n.value


def batch_compile_check(motifs, key_bytes=4, tier=0) -> int:
    """Compile the batched module a count batch of synth.Motif-like objects
    launches under ``tier`` (no device)."""
    descs = (N.MotifDesc * len(motifs))()
    keep = []
    for i, m in enumerate(motifs):
        d, k = motif_desc_of(m)
        descs[i] = d
        keep.append(k)
    n = ctypes.c_int64(0)
    N.check(N.lib().tm_batch_compile_check(descs, len(motifs), int(tier), key_bytes, ctypes.byref(n)))
    return n.value


class Context:
    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        N.check(N.lib().tm_create(int(device), ctypes.byref(h)))
        self._h = h
        self.device = device
        self._servers = weakref.WeakSet()  # servers use the context until they stop

    def close(self):
        if self._h:
            for srv in list(self._servers):
                srv.stop()
            N.lib().tm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- params
    def set_param(self, param: int, value: int):
        N.check(N.lib().tm_set_param(self._h, int(param), int(value)))

    def get_param(self, param: int) -> int:
        v = ctypes.c_int64()
        N.check(N.lib().tm_get_param(self._h, int(param), ctypes.byref(v)))
        return v.value

    def last_kernel_ms(self):
        ms = ctypes.c_double()
        n = ctypes.c_int32()
        N.check(N.lib().tm_last_kernel_ms(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def last_launch(self):
        """(root chunk, split flag, tuned flag) of the last mining call."""
        return self.last_launch_full()[:3]

    def last_trace(self) -> np.ndarray:
        """Samples of the last mining launch taken with TM_PARAM_TRACE_US > 0:
        int64[n, 8] rows of (ns since queued, chunks taken, chunks, busy
        wavefronts, waiting wavefronts, donated items waiting, done, roots
        handed to waiting wavefronts)."""
        n = ctypes.c_int64(0)
        N.check(N.lib().tm_last_trace(self._h, None, 0, ctypes.byref(n)))
        out = np.zeros((n.value, 8), np.int64)
        N.check(N.lib().tm_last_trace(self._h, _ptr(out), n.value, ctypes.byref(n)))
        return out[:n.value]

    def last_launch_full(self):
        """(root chunk, split flag, tuned flag, smallest split window, smallest
        window counted in closed form) of the last mining call."""
        r, sp, sm, lm, tu = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        N.check(N.lib().tm_last_launch(self._h, ctypes.byref(r), ctypes.byref(sp), ctypes.byref(sm),
                                       ctypes.byref(lm), ctypes.byref(tu)))
        return r.value, sp.value, tu.value, sm.value, lm.value

    def tune_save(self, path):
        N.check(N.lib().tm_tune_save(self._h, os.fsencode(path)))

    def tune_load(self, path):
        N.check(N.lib().tm_tune_load(self._h, os.fsencode(path)))

    def tune_clear(self) -> int:
        n = ctypes.c_int64()
        N.check(N.lib().tm_tune_clear(self._h, ctypes.byref(n)))
        return n.value

    # ---- graph / motif
    def load_graph(self, n_nodes, src, dst, t, w=None) -> Graph:
        s = _np(src, np.int32)
        d = _np(dst, np.int32)
        tt = _np(t, np.int64)
        ww = _np(w, np.float32)
        h = ctypes.c_void_p()
        N.check(N.lib().tm_load_graph(self._h, int(n_nodes), int(s.size), _ptr(s), _ptr(d), _ptr(tt), _ptr(ww), 0,
                                      ctypes.byref(h)))
        return Graph(self, h)

    def load_synth(self, g) -> Graph:
        dg = self.load_graph(g.n, g.src, g.dst, g.t, g.w)
        if getattr(g, "labels", None) is not None:
            dg.set_node_labels(g.labels)
        if getattr(g, "edge_labels", None) is not None:
            dg.set_edge_labels(g.edge_labels)
        return dg

    def compile_motif(self, edges, delta, gap=None, pred_edge=-1, pred_op=0, pred_theta=0.0,
                      n_nodes=None, anti=None, node_labels=None, node_label_hi=None, preds=None,
                      edge_labels=None) -> Motif:
        d, keep = make_desc(edges, delta, gap, pred_edge, pred_op, pred_theta, n_nodes, anti, node_labels,
                            node_label_hi, preds, edge_labels)
        h = ctypes.c_void_p()
        N.check(N.lib().tm_compile_motif(self._h, ctypes.byref(d), ctypes.byref(h)))
        return Motif(self, h, d.n_edges)

    def compile(self, m) -> Motif:
        """Compile a synth.Motif-like object."""
        return self.compile_motif(m.edges, m.delta, None if m.gap is None else m.gaps(), m.pred_edge, m.pred_op,
                                  m.pred_theta, anti=getattr(m, "anti", None),
                                  node_labels=getattr(m, "node_labels", None),
                                  node_label_hi=getattr(m, "node_label_hi", None), preds=getattr(m, "preds", None),
                                  edge_labels=getattr(m, "edge_labels", None))

    # ---- mining
    def count(self, g: Graph, m: Motif, t_lo=None, t_hi=None, stream=None) -> int:
        rr = _range(t_lo, t_hi)
        out = ctypes.c_uint64()
        N.check(N.lib().tm_count(self._h, g.handle, m.handle, None if rr is None else ctypes.byref(rr),
                                 _stream_handle(stream), ctypes.byref(out)))
        return out.value

    def work_stats(self, g: Graph, m: Motif, t_lo=None, t_hi=None, stream=None, leaf=False) -> dict:
        """The method's work counters (as the oracle's); with leaf=True also
        the counters of the closed-form last-level counts."""
        rr = _range(t_lo, t_hi)
        st = np.zeros(9, np.uint64)
        N.check(N.lib().tm_work_stats(self._h, g.handle, m.handle, None if rr is None else ctypes.byref(rr),
                                      _stream_handle(stream), _ptr(st)))
        keys = ("roots", "windows", "probes", "visits", "pred_visits", "matches")
        if leaf:
            keys += ("leaf_counted", "leaf_counted_visits", "leaf_count_reads")
        return {k: int(v) for k, v in zip(keys, st)}

    def enumerate_into(self, g: Graph, m: Motif, out_ptr: int, capacity: int, t_lo=None, t_hi=None,
                       stream=None):
        """Enumerate into caller-owned device memory; returns (status, n)."""
        rr = _range(t_lo, t_hi)
        n = ctypes.c_uint64()
        st = N.lib().tm_enumerate(self._h, g.handle, m.handle, None if rr is None else ctypes.byref(rr),
                                  _stream_handle(stream), ctypes.c_void_p(out_ptr) if out_ptr else None,
                                  int(capacity), ctypes.byref(n))
        if st not in (N.TM_OK, N.TM_E_CAPACITY):
            N.check(st)
        return st, n.value

    def enumerate(self, g: Graph, m: Motif, t_lo=None, t_hi=None, stream=None, capacity=None):
        """All instances as a device int64 tensor [count, l] (rows grouped by
        root chunk; the order inside a chunk is unspecified)."""
        import torch
        if capacity is None:
            _, capacity = self.enumerate_into(g, m, 0, 0, t_lo, t_hi, stream)
        out = torch.empty((max(int(capacity), 1), m.l), dtype=torch.int64, device=f"cuda:{self.device}")
        st, n = self.enumerate_into(g, m, out.data_ptr(), int(capacity), t_lo, t_hi, stream)
        if st == N.TM_E_CAPACITY:
            raise N.NativeError(st, f"capacity {capacity} < {n}")
        return out[:n]

    def count_batch(self, g: Graph, motifs: Sequence[Motif], ranges=None, stream=None, allow_cancel=False):
        """Counts of all queries in one launch. With allow_cancel, queries over
        the work budget give None instead of raising TM_E_CANCELLED."""
        q = len(motifs)
        arr = (ctypes.c_void_p * max(q, 1))(*[mm.handle.value if hasattr(mm.handle, "value") else mm.handle
                                              for mm in motifs])
        rr = None
        if ranges is not None:
            rr = (N.RootRange * q)(*[N.RootRange(I64_MIN if a is None else int(a), I64_MAX if b is None else int(b))
                                     for a, b in ranges])
        out = np.zeros(max(q, 1), np.uint64)
        st = N.lib().tm_count_batch(self._h, g.handle, q, arr, rr, _stream_handle(stream), _ptr(out))
        if st == N.TM_E_CANCELLED and allow_cancel:
            return [None if int(x) == 2**64 - 1 else int(x) for x in out[:q]]
        N.check(st)
        return [int(x) for x in out[:q]]

    def count_batch_noalloc(self, g: Graph, motifs: Sequence[Motif], ranges=None, stream=None):
        """count_batch on the library's device scratch (no device allocation);
        the batched kernel of these motifs must be loaded already."""
        q = len(motifs)
        arr = (ctypes.c_void_p * max(q, 1))(*[mm.handle.value if hasattr(mm.handle, "value") else mm.handle
                                              for mm in motifs])
        rr = None
        if ranges is not None:
            rr = (N.RootRange * q)(*[N.RootRange(I64_MIN if a is None else int(a), I64_MAX if b is None else int(b))
                                     for a, b in ranges])
        out = np.zeros(max(q, 1), np.uint64)
        N.check(N.lib().tm_count_batch_noalloc(self._h, g.handle, q, arr, rr, _stream_handle(stream), _ptr(out)))
        return [int(x) for x in out[:q]]


class _DeviceRows:
    """Device memory the server owns, exposed to torch without a copy."""

    def __init__(self, ptr, n, l):
        self.__cuda_array_interface__ = {"data": (int(ptr), False), "shape": (int(n), int(l)),
                                         "typestr": "<i8", "version": 2, "strides": None}


class Server:
    """Continuous-batching query server over one resident graph (tm_server_*).

    tier: 0 specialised kernels, 1 table-driven, 2 table-driven batches with
    the count queries over ``probe_budget`` steps run again on specialised
    kernels compiled in the background (results then carry ``kernel_tier``
    and ``probed``)."""

    def __init__(self, ctx: Context, g: Graph, stream_slots=2, max_batch=64, enum_pool_bytes=1 << 30,
                 queue_capacity=1 << 16, tier=1, tune_path=None, work_budget=0, probe_budget=0):
        self._tune_path = None if tune_path is None else os.fsencode(tune_path)  # kept alive for the call
        cfg = N.ServerCfg(int(stream_slots), int(max_batch), int(enum_pool_bytes), int(queue_capacity), int(tier),
                          int(work_budget), self._tune_path, int(probe_budget))
        h = ctypes.c_void_p()
        N.check(N.lib().tm_server_start(ctx._h, g.handle, ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._ctx = ctx
        self._g = g
        ctx._servers.add(self)

    def submit(self, motif, t_lo=None, t_hi=None, enumerate=False, tag=0, work_budget=0) -> int:
        """Submit a synth.Motif-like query; returns its ticket."""
        d, keep = motif_desc_of(motif)
        q = N.Query()
        q.motif = d
        q.has_range = 0 if (t_lo is None and t_hi is None) else 1
        q.range = N.RootRange(I64_MIN if t_lo is None else int(t_lo), I64_MAX if t_hi is None else int(t_hi))
        q.enumerate = 1 if enumerate else 0
        q.tag = int(tag)
        q.work_budget = int(work_budget)
        t = ctypes.c_uint64()
        N.check(N.lib().tm_submit_query(self._h, ctypes.byref(q), ctypes.byref(t)))
        return t.value

    def poll(self, max_results=256, timeout_ms=0):
        buf = (N.Result * max_results)()
        n = ctypes.c_int32()
        N.check(N.lib().tm_poll(self._h, buf, int(max_results), ctypes.byref(n), int(timeout_ms)))
        out = []
        for r in buf[:n.value]:
            out.append({"ticket": r.ticket, "tag": r.tag, "status": r.status, "count": r.count,
                        "rows": r.rows, "n_rows": r.n_rows, "n_edges": r.n_edges,
                        "t_arrival_ns": r.t_arrival_ns, "t_admit_ns": r.t_admit_ns,
                        "t_launch_ns": r.t_launch_ns, "t_done_ns": r.t_done_ns,
                        "error": r.error.decode(errors="replace"), "kernel_tier": r.kernel_tier,
                        "probed": bool(r.probed)})
        return out

    def rows(self, result):
        """The result's rows as a torch tensor (a copy; release the ticket after)."""
        import torch
        if not result["rows"] or result["n_rows"] == 0:
            return torch.zeros((0, result["n_edges"]), dtype=torch.int64, device=f"cuda:{self._ctx.device}")
        dev = torch.device(f"cuda:{self._ctx.device}")
        view = torch.as_tensor(_DeviceRows(result["rows"], result["n_rows"], result["n_edges"]), device=dev)
        out = view.clone()
        # the copy must be done before release() hands the memory to another result
        torch.cuda.current_stream(dev).synchronize()
        return out

    def release(self, ticket):
        N.check(N.lib().tm_release(self._h, ctypes.c_uint64(int(ticket))))

    def stats(self):
        a, b, c = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        N.check(N.lib().tm_server_stats(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return {"served": a.value, "batches": b.value, "pending": c.value}

    def stop(self):
        if self._h:
            N.check(N.lib().tm_server_stop(self._h))
            self._h = None

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass


def tail_summary(samples) -> dict:
    """Load balance of one sampled launch: when its root-chunk queue drained
    and what ran after that. Times from the first sample with a wavefront at
    work (or a chunk taken) to the first sample after the kernel ended, so
    they carry the sampling period as error."""
    s = np.asarray(samples)
    if s.shape[0] == 0:
        return {}
    started = np.nonzero((s[:, 1] > 0) | (s[:, 3] > 0))[0]
    t_start = int(s[started[0], 0]) if started.size else int(s[0, 0])
    t_end = int(s[-1, 0])
    drained = np.nonzero(s[:, 1] >= s[:, 2])[0]
    t_drain = int(s[drained[0], 0]) if drained.size else t_end
    tail = s[(s[:, 0] >= t_drain) & (s[:, 6] == 0)]
    span = max(t_end - t_start, 1)
    busy_after = float(tail[:, 3].mean()) if tail.shape[0] else 0.0
    peak = int(s[:, 3].max())
    tail_frac = (t_end - t_drain) / span
    return {"samples": int(s.shape[0]), "run_ms": span / 1e6, "drain_ms": (t_drain - t_start) / 1e6,
            "tail_ms": (t_end - t_drain) / 1e6, "tail_frac": tail_frac,
            "busy_after_drain_mean": busy_after, "busy_peak": peak,
            # share of the launch's wavefront time spent idle after the queue drained
            "idle_share": tail_frac * (1.0 - busy_after / peak) if peak else 0.0,
            "roots_handed": int(s[-1, 7]) if s.shape[1] > 7 else 0}
