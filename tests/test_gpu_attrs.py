"""General attribute constraints on the GPU against the oracle, both kernel
tiers (Sec. 2.1: node and edge attributes a query constrains; Sec. 5.4.1:
generated checks when a vertex or edge is newly matched): several weight
predicates (also intervals on one edge), vertex label ranges and edge label
ranges, alone and together with gaps and anti-edges.

Exact comparisons throughout: counts, sorted instance sets and work counters.
Cases put each kind of constraint on the root, a middle level and the last
level (where an edge label or predicate turns the closed-form count off), on
a whole-edge-list level, and on levels the wavefront-cooperative scan reads.
Also mixed batches, the serving loop, random small graphs, a graph without
edge labels, and the full-size wiki-shaped graph.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from paper_2310_02800_amd import _native as N
from paper_2310_02800_amd import api, synth

pytestmark = pytest.mark.gpu
Motif = synth.Motif
GE, GT, LE, LT = synth.PRED_GE, synth.PRED_GT, synth.PRED_LE, synth.PRED_LT


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def sorted_rows(a):
    a = a.cpu().numpy() if hasattr(a, "cpu") else np.asarray(a)
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a[np.lexsort(a.T[::-1])] if a.ndim == 2 and a.shape[0] else a


def same_rows(a, b):
    a, b = sorted_rows(a), sorted_rows(b)
    return a.shape[0] == b.shape[0] and (a.shape[0] == 0 or np.array_equal(a, b))


# tiny graph (1,000 nodes, 20,000 edges, time span 1e6) with 4 node labels
# and 3 edge labels
TINY_CASES = [
    Motif(synth.FOUR_CYCLE, 86_400, preds=[(1, GE, 0.5), (1, LT, 2.5)]),                # interval on one edge
    Motif(synth.TRIANGLE, 20_000, edge_labels=[(1, 2), (-1, -1), (-1, -1)]),             # root edge label
    Motif(synth.TRIANGLE, 20_000, edge_labels=[(-1, -1), (0, 0), (1, 2)]),               # last level: closed form off
    Motif(synth.OUT_STAR3, 3000, preds=[(2, GT, 0.8)]),                                  # predicate on the last level
    Motif(synth.OUT_STAR3, 3000, preds=[(0, LE, 3.0), (1, GE, 0.3)]),                    # above the last level
    Motif(synth.OUT_STAR3, 3000, node_labels=[0, -1, -1, 1], node_label_hi=[2, -1, -1, 3]),  # label ranges
    Motif([(0, 1), (1, 2), (2, 3)], 10_000, node_labels=[-1, 1, 0, -1], node_label_hi=[-1, 3, 1, -1],
          edge_labels=[(-1, -1), (0, 1), (-1, -1)], preds=[(0, GE, 0.4), (2, LT, 1.5)]),  # everything
    Motif([(0, 1), (2, 3)], 200, edge_labels=[(0, 1), (2, 2)], preds=[(1, GE, 0.2)]),    # whole edge list level
    Motif(synth.FOUR_CYCLE, 86_400, gap=[30_000] * 3, preds=[(3, GE, 0.5)], edge_labels=[(-1, -1)] * 3 + [(0, 1)],
          anti=[(2, 0, 2, 20_000)]),                                                     # with gaps and an anti-edge
    Motif(synth.FOUR_CYCLE, 86_400, pred_edge=0, pred_op=GE, pred_theta=0.3, preds=[(0, LT, 3.0), (2, GE, 0.3)]),
]

# a dense graph (12 nodes) whose last-level windows are wide: the
# wavefront-cooperative scan and the closed form both run
DENSE_CASES = [
    Motif([(0, 1), (0, 2), (0, 3)], 300, edge_labels=[(-1, -1), (-1, -1), (0, 1)]),  # label on the coop level
    Motif([(0, 1), (0, 2), (0, 3)], 300, preds=[(2, GE, 0.5), (2, LE, 2.0)]),        # interval on the coop level
    Motif([(0, 1), (0, 2), (0, 3)], 300, edge_labels=[(1, 2), (-1, -1), (-1, -1)],
          node_labels=[0, -1, -1, -1], node_label_hi=[1, -1, -1, -1]),               # above: closed form stays on
    Motif(synth.TRIANGLE, 600, preds=[(1, LT, 1.0)]),                                # both ends bound, pred above
]


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    yield c
    c.close()


def attributed(g, seed):
    g = synth.with_labels(g, synth.node_labels(seed, g.n, 4))
    return synth.with_edge_labels(g, synth.edge_labels(seed + 1, g.m, 3))


@pytest.fixture(scope="module")
def tiny():
    return attributed(synth.tiny_graph(0), 31)


@pytest.fixture(scope="module")
def tiny_g(ctx, tiny):
    dg = ctx.load_synth(tiny)
    inf = dg.info()
    assert inf["has_labels"] == 1 and inf["has_edge_labels"] == 1
    return dg


@pytest.fixture(scope="module")
def tiny_og(tiny):
    return oracle.OracleGraph.from_graph(tiny)


@pytest.fixture(scope="module")
def dense():
    g = synth.random_graph(np.random.Generator(np.random.PCG64(23)), 12, 30_000, 20_000, self_loops=True)
    return attributed(g, 41)


@pytest.fixture(scope="module")
def dense_g(ctx, dense):
    return ctx.load_synth(dense)


@pytest.fixture(scope="module")
def dense_og(dense):
    return oracle.OracleGraph.from_graph(dense)


def with_params(ctx, values):
    old = {p: ctx.get_param(p) for p in values}
    for p, v in values.items():
        ctx.set_param(p, v)
    return old


@pytest.mark.parametrize("tier", [0, 1])
@pytest.mark.parametrize("split", [0, 1])
@pytest.mark.parametrize("k", range(len(TINY_CASES)))
def test_tiny_counts_rows_and_counters(ctx, tiny_g, tiny_og, k, split, tier):
    mot = TINY_CASES[k]
    old = with_params(ctx, {N.TM_PARAM_SPLIT: split, N.TM_PARAM_TIER: tier})
    try:
        mm = ctx.compile(mot)
        want, st = oracle.count(tiny_og, mot, nthreads=8, list_rule=1, with_stats=True)
        say("attr case", k, "tier", tier, "split", split, mot.edges, "count", want)
        assert want > 0
        assert ctx.count(tiny_g, mm) == want
        assert ctx.work_stats(tiny_g, mm) == st
        assert same_rows(ctx.enumerate(tiny_g, mm), oracle.enumerate(tiny_og, mot))
    finally:
        with_params(ctx, old)


@pytest.mark.parametrize("tier", [0, 1])
@pytest.mark.parametrize("k", range(len(DENSE_CASES)))
def test_dense_wide_windows(ctx, dense_g, dense_og, k, tier):
    mot = DENSE_CASES[k]
    old = with_params(ctx, {N.TM_PARAM_LEAF_MIN: 32, N.TM_PARAM_TIER: tier})
    try:
        mm = ctx.compile(mot)
        want, st = oracle.count(dense_og, mot, nthreads=8, list_rule=1, with_stats=True)
        say("dense attr case", k, "tier", tier, mot.edges, "count", want)
        assert want > 0
        assert ctx.count(dense_g, mm) == want
        ws = ctx.work_stats(dense_g, mm, leaf=True)
        assert {key: ws[key] for key in st} == st
        if k in (0, 1):
            assert ws["leaf_counted"] == 0  # a constraint on the last level: scanned
        else:
            assert ws["leaf_counted"] > 0
        lo, hi = 5_000, 5_600
        rows = ctx.enumerate(dense_g, mm, t_lo=lo, t_hi=hi)
        assert same_rows(rows, oracle.enumerate(dense_og, mot, t_lo=lo, t_hi=hi))
    finally:
        with_params(ctx, old)


@pytest.mark.parametrize("tier", [0, 1])
def test_batch_mixes_constrained_and_plain(ctx, tiny_g, tiny_og, tier):
    qs = list(TINY_CASES) + [Motif(m.edges, m.delta, gap=m.gap) for m in TINY_CASES[:4]]
    old = with_params(ctx, {N.TM_PARAM_TIER: tier, N.TM_PARAM_SPLIT: 0})
    try:
        handles = [ctx.compile(m) for m in qs]
        want = [oracle.count(tiny_og, m, nthreads=8) for m in qs]
        for split in (0, 1):
            ctx.set_param(N.TM_PARAM_SPLIT, split)
            say("attr batch tier", tier, "split", split)
            assert ctx.count_batch(tiny_g, handles) == want
    finally:
        with_params(ctx, old)


def test_served_constrained_queries(ctx, tiny_g, tiny_og):
    srv = api.Server(ctx, tiny_g, stream_slots=2, max_batch=8, enum_pool_bytes=64 << 20, tier=1)
    try:
        for i, m in enumerate(TINY_CASES):
            srv.submit(m, enumerate=(i % 2 == 1), tag=i)
        got = {}
        for _ in range(600):
            for r in srv.poll(64, timeout_ms=200):
                got[r["tag"]] = (r, srv.rows(r) if r["rows"] else None)
                srv.release(r["ticket"])
            if len(got) == len(TINY_CASES):
                break
    finally:
        srv.stop()
    assert len(got) == len(TINY_CASES)
    for i, m in enumerate(TINY_CASES):
        r, rows = got[i]
        assert r["status"] == N.TM_OK
        want = oracle.enumerate(tiny_og, m)
        assert r["count"] == want.shape[0], (i, m)
        if i % 2 == 1:
            assert same_rows(rows, want)


@pytest.mark.parametrize("seed", [0, 1])
def test_random_small_graphs(ctx, seed):
    """60 random cases per seed: tiny graphs with node and edge labels and
    random constraints of every kind, count and enumeration, both tiers."""
    rng = np.random.Generator(np.random.PCG64(700 + seed))
    nonzero = 0
    for case in range(60):
        l = int(rng.integers(1, 5))
        k = int(rng.integers(2, min(5, l + 1) + 1))
        me = synth.random_motif(rng, l, k)
        n, m, t_max = int(rng.integers(3, 7)), int(rng.integers(10, 60)), int(rng.integers(10, 40))
        g = synth.random_graph(rng, n, m, t_max)
        g = synth.with_edge_labels(synth.with_labels(g, rng.integers(0, 2, n)), rng.integers(0, 2, m))
        mot = Motif(me, int(rng.integers(t_max // 2, t_max + 2)))
        if rng.random() < 0.6:
            lo = [int(x) for x in rng.integers(-1, 2, mot.k)]
            mot.node_labels = lo
            mot.node_label_hi = [x + int(rng.integers(0, 2)) if x >= 0 else -1 for x in lo]
        if rng.random() < 0.6:
            el = []
            for _ in range(l):
                a = int(rng.integers(-1, 2))
                el.append((a, a + int(rng.integers(0, 2)) if a >= 0 else -1))
            mot.edge_labels = el
        if rng.random() < 0.6:
            mot.preds = [(int(rng.integers(0, l)), int(rng.integers(0, 4)), float(np.float32(rng.lognormal(0, 0.5))))
                         for _ in range(int(rng.integers(1, 4)))]
        dg = ctx.load_synth(g)
        og = oracle.OracleGraph.from_graph(g)
        want = oracle.enumerate(og, mot)
        nonzero += want.shape[0] > 0
        for tier in (0, 1):
            old = with_params(ctx, {N.TM_PARAM_TIER: tier})
            try:
                mm = ctx.compile(mot)
                assert ctx.count(dg, mm) == want.shape[0], (seed, case, tier, mot)
                assert same_rows(ctx.enumerate(dg, mm), want)
            finally:
                with_params(ctx, old)
    assert nonzero >= 10, nonzero


def test_edge_labels_required_but_missing(ctx):
    g = synth.tiny_graph(0)
    dg = ctx.load_synth(g)
    assert dg.info()["has_edge_labels"] == 0
    with pytest.raises(N.NativeError) as ei:
        ctx.count(dg, ctx.compile(Motif(synth.TRIANGLE, 100, edge_labels=[(0, 0), (-1, -1), (-1, -1)])))
    assert ei.value.status == N.TM_E_INVALID
    with pytest.raises(N.NativeError):
        dg.set_edge_labels(np.full(g.m, -1, np.int32))
    with pytest.raises(N.NativeError):  # empty range
        ctx.compile(Motif(synth.TRIANGLE, 100, edge_labels=[(2, 1), (-1, -1), (-1, -1)]))
    with pytest.raises(N.NativeError):  # predicate on a missing edge
        ctx.compile(Motif(synth.TRIANGLE, 100, preds=[(3, GE, 1.0)]))


def test_edge_labels_follow_a_resorted_input(ctx, tiny):
    """Edge labels are given in input order; an input out of time order is
    sorted by the library and the labels must move with their edges."""
    rng = np.random.Generator(np.random.PCG64(9))
    perm = rng.permutation(tiny.m)
    dg = ctx.load_graph(tiny.n, tiny.src[perm], tiny.dst[perm], tiny.t[perm], tiny.w[perm])
    dg.set_node_labels(tiny.labels)
    dg.set_edge_labels(tiny.edge_labels[perm])
    order = dg.edge_order()
    og = oracle.OracleGraph(tiny.n, tiny.src[perm][order], tiny.dst[perm][order], tiny.t[perm][order],
                            tiny.w[perm][order], tiny.labels, tiny.edge_labels[perm][order])
    for mot in TINY_CASES[:3]:
        assert ctx.count(dg, ctx.compile(mot)) == oracle.count(og, mot, nthreads=8)


WIKI_CASES = [
    Motif(synth.FOUR_CYCLE, 86_400, node_labels=[0, 1, 0, 1], node_label_hi=[1, 2, 1, 2],
          edge_labels=[(0, 1), (-1, -1), (0, 1), (-1, -1)]),
    Motif(synth.FOUR_CYCLE, 86_400, preds=[(0, GE, 0.5), (0, LT, 2.0), (3, GE, 1.0)]),
    Motif(synth.OUT_STAR3, 3600, edge_labels=[(-1, -1), (-1, -1), (2, 2)], preds=[(1, LE, 1.5)]),
    Motif(synth.TRIANGLE, 86_400, node_labels=[1, -1, -1], node_label_hi=[2, -1, -1], preds=[(2, GT, 0.7)]),
]


def test_wiki_full_counts(ctx):
    say("generating wiki-shaped graph")
    g = attributed(synth.wiki_graph(), 51)
    og = oracle.OracleGraph.from_graph(g)
    dg = ctx.load_synth(g)
    want = []
    for mot in WIKI_CASES:
        want.append(oracle.count(og, mot, nthreads=16))
        say("wiki attrs", mot.edges, "oracle", want[-1])
        assert want[-1] > 0
        assert ctx.count(dg, ctx.compile(mot)) == want[-1]
    old = with_params(ctx, {N.TM_PARAM_TIER: 1})
    try:
        assert ctx.count_batch(dg, [ctx.compile(m) for m in WIKI_CASES]) == want
    finally:
        with_params(ctx, old)
