"""The seeded input generators produce the workloads they describe: sizes,
time order and span, degree skew, per-source spacing, query mixes. The GPU
tests and the bench take these graphs and query sets as the stand-ins for
the paper's datasets, so their recipe is pinned here (CPU only)."""
from __future__ import annotations

import math

import numpy as np
import pytest

from paper_2310_02800_amd import synth


def harmonic(n):
    return float(np.sum(1.0 / np.arange(1, n + 1, dtype=np.float64)))


def check_time_ordered(g):
    assert g.src.size == g.dst.size == g.t.size == g.m
    assert np.all(np.diff(g.t) >= 0)
    assert g.src.min() >= 0 and g.dst.min() >= 0 and max(g.src.max(), g.dst.max()) < g.n
    assert not np.any(g.src == g.dst)  # no self-loops in the power-law graphs


def test_tiny_graph_recipe():
    g = synth.tiny_graph(0)
    check_time_ordered(g)
    assert (g.n, g.m) == (1000, 20_000)
    assert g.t.min() >= 0 and g.t.max() < 1_000_000
    assert np.any(np.diff(g.t) == 0)  # ties occur
    assert g.w.dtype == np.float32 and np.all(g.w > 0)
    lw = np.log(g.w.astype(np.float64))
    assert abs(lw.mean()) < 0.05 and abs(lw.std() - 1.0) < 0.05  # log-normal(0, 1)
    deg = np.bincount(g.src, minlength=g.n) + np.bincount(g.dst, minlength=g.n)
    assert deg.max() > 10 * deg.mean()  # power law (exponent 2.1): a few nodes hold many edges


def test_wiki_graph_recipe():
    g = synth.wiki_graph()
    check_time_ordered(g)
    assert (g.n, g.m) == (1_100_000, 7_800_000)
    assert g.t.min() >= 0 and g.t.max() < 2e8 and g.t.max() - g.t.min() > 0.99 * 2e8
    out_deg = np.bincount(g.src, minlength=g.n)
    in_deg = np.bincount(g.dst, minlength=g.n)
    # expected top degree 1e5 in each direction (Chung-Lu with w_i = 1/(i + i0))
    assert 0.8e5 < out_deg.max() < 1.25e5 and 0.8e5 < in_deg.max() < 1.25e5
    assert np.argmax(out_deg) == 0 and np.argmax(in_deg) == 0
    assert g.w.dtype == np.float32 and np.all(g.w > 0)


def test_skew_graph_recipe_small():
    n, m, span = 50_000, 300_000, 3_000_000
    g = synth.skew_graph(seed=6, n=n, m=m, span=span)
    check_time_ordered(g)
    assert g.t.min() >= 0 and g.t.max() <= span
    # Zipf weights w_i = 1/(i + 1): the top node's expected out-degree is m / H(n)
    top = np.bincount(g.src, minlength=n).max()
    assert 0.8 < top / (m / harmonic(n)) < 1.25
    # per source, consecutive edges 1-20 s apart
    order = np.lexsort((g.t, g.src))
    s, t = g.src[order], g.t[order]
    same = s[1:] == s[:-1]
    gaps = np.diff(t)[same]
    assert gaps.min() >= 1 and gaps.max() <= 20
    assert abs(gaps.mean() - 10.5) < 0.1


def motif_order_connected(edges):
    seen = {edges[0][0], edges[0][1]}
    if edges[0] != (0, 1):
        return False
    for a, b in edges[1:]:
        if a == b or (a not in seen and b not in seen):
            return False
        new = [x for x in (a, b) if x not in seen]
        if len(new) > 1 or (new and new[0] != len(seen)):
            return False
        seen.update(new)
    return True


def test_batch_queries_recipe():
    qs = synth.batch_queries()
    assert len(qs) == 64
    for i, q in enumerate(qs):
        assert 3 <= q.l <= 6 and 3 <= q.k <= min(5, q.l + 1)
        assert len({x for e in q.edges for x in e}) == q.k
        assert motif_order_connected([tuple(e) for e in q.edges])
        assert 600 <= q.delta <= 86_400
        assert (q.pred_edge >= 0) == (i % 2 == 1)
        if q.pred_edge >= 0:
            assert 0 <= q.pred_edge < q.l and q.pred_op in (synth.PRED_GE, synth.PRED_LT)
    # delta log-uniform: about half of the queries below the geometric mean
    below = sum(q.delta < math.sqrt(600 * 86_400) for q in qs)
    assert 20 <= below <= 44


def test_serve_queries_recipe():
    t_min, t_max = 0, 200_000_000
    qs = synth.serve_queries(t_min, t_max)
    assert len(qs) == 10_000
    enum = sum(q.enumerate for q in qs)
    assert 900 <= enum <= 1100  # 10% enumerations
    arr = np.array([q.arrival for q in qs])
    assert np.all(np.diff(arr) > 0)
    assert abs(np.mean(np.diff(arr)) - 1.0) < 0.05  # unit-rate Poisson arrivals
    frac = np.array([(q.t_hi - q.t_lo) / (t_max - t_min) for q in qs])
    assert frac.min() >= 0.0099 and frac.max() <= 1.0
    assert all(t_min <= q.t_lo <= q.t_hi <= t_max for q in qs)
    for q in qs[:500]:
        m = q.motif
        assert 3 <= m.l <= 6 and 600 <= m.delta <= 86_400
        assert motif_order_connected([tuple(e) for e in m.edges])


@pytest.mark.parametrize("n_labels", [2, 4])
def test_labels_recipe(n_labels):
    lab = synth.node_labels(2, 100_000, n_labels)
    assert lab.dtype == np.int32 and lab.min() == 0 and lab.max() == n_labels - 1
    share = np.bincount(lab) / lab.size
    assert np.all(np.abs(share - 1.0 / n_labels) < 0.01)
    el = synth.edge_labels(3, 100_000, 3)
    assert el.min() == 0 and el.max() == 2
