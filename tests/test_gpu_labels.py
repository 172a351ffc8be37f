"""Vertex labels (Sec. 5.4.1) on the GPU against the oracle, both kernel tiers.

Exact comparisons throughout: counts, sorted instance sets and work counters.
Cases: the paper's query shape (a 4-cycle with two nodes of each of two
labels), a labelled root node, a labelled node first bound on the last level
(which turns the closed-form count off) and on a middle level, two new nodes
bound by a whole-edge-list level, a star pinned at the hub (its centre's
label held by that node alone), and labels with gaps, a predicate and an
anti-edge. Also mixed batches, the serving loop, a graph without labels, and
the full-size wiki-shaped graph.
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


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def sorted_rows(a):
    a = a.cpu().numpy() if hasattr(a, "cpu") else np.asarray(a)
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a[np.lexsort(a.T[::-1])] if a.ndim == 2 and a.shape[0] else a


def same_rows(a, b):
    a, b = sorted_rows(a), sorted_rows(b)
    return a.shape[0] == b.shape[0] and (a.shape[0] == 0 or np.array_equal(a, b))


# tiny graph (1,000 nodes, 20,000 edges, time span 1e6) with 4 random labels
TINY_CASES = [
    Motif(synth.FOUR_CYCLE, 86_400, node_labels=[0, 1, 0, 1]),          # the paper's query shape
    Motif(synth.TRIANGLE, 20_000, node_labels=[2, -1, -1]),             # root node only
    Motif(synth.OUT_STAR3, 3000, node_labels=[-1, -1, -1, 3]),          # new node of the last level
    Motif([(0, 1), (1, 2), (2, 3)], 10_000, node_labels=[-1, -1, 1, -1]),  # new node of a middle level
    Motif([(0, 1), (2, 3)], 200, node_labels=[-1, -1, 0, 2]),           # two new nodes, whole edge list
    Motif([(0, 1), (1, 2), (0, 2), (2, 3)], 50_000, gap=[20_000] * 3, pred_edge=2, pred_op=synth.PRED_GE,
          pred_theta=0.5, anti=[(3, 0, 3, 10_000)], node_labels=[1, -1, 0, 2]),  # with gaps, predicate, anti-edge
]

# dense multigraph (12 nodes, 30,000 edges over 20,000) with 3 labels
DENSE_CASES = [
    Motif([(0, 1), (0, 2), (0, 3)], 300, node_labels=[-1, -1, -1, 1]),  # labelled new node: closed form off
    Motif([(0, 1), (0, 2), (0, 3)], 300, node_labels=[0, 1, -1, -1]),   # labels above the last level
    Motif(synth.TRIANGLE, 600, node_labels=[-1, -1, 2]),               # last level binds nothing new
]


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def tiny():
    g = synth.tiny_graph(0)
    return synth.with_labels(g, synth.node_labels(11, g.n, 4))


@pytest.fixture(scope="module")
def tiny_g(ctx, tiny):
    dg = ctx.load_synth(tiny)
    assert dg.info()["has_labels"] == 1
    return dg


@pytest.fixture(scope="module")
def tiny_og(tiny):
    return oracle.OracleGraph.from_graph(tiny)


@pytest.fixture(scope="module")
def dense():
    g = synth.random_graph(np.random.Generator(np.random.PCG64(21)), 12, 30_000, 20_000, self_loops=True)
    return synth.with_labels(g, synth.node_labels(12, g.n, 3))


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
        say("tiny case", k, "tier", tier, "split", split, mot.edges, mot.node_labels, "count", want)
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
        say("dense case", k, "tier", tier, mot.edges, mot.node_labels, "count", want)
        assert ctx.count(dense_g, mm) == want
        ws = ctx.work_stats(dense_g, mm, leaf=True)
        assert {key: ws[key] for key in st} == st
        if k == 0:
            assert ws["leaf_counted"] == 0
        else:
            assert ws["leaf_counted"] > 0
        lo, hi = 5_000, 5_600
        rows = ctx.enumerate(dense_g, mm, t_lo=lo, t_hi=hi)
        assert same_rows(rows, oracle.enumerate(dense_og, mot, t_lo=lo, t_hi=hi))
    finally:
        with_params(ctx, old)


def test_star_pinned_at_the_hub(ctx, tiny):
    """A 3-edge out-star whose centre must be the highest out-degree node: a
    label that node alone carries."""
    hub = int(np.argmax(np.bincount(tiny.src, minlength=tiny.n)))
    lab = np.zeros(tiny.n, np.int32)
    lab[hub] = 1
    g = synth.with_labels(tiny, lab)
    dg = ctx.load_synth(g)
    og = oracle.OracleGraph.from_graph(g)
    mot = Motif(synth.OUT_STAR3, 3000, node_labels=[1, -1, -1, -1])
    want = oracle.count(og, mot, nthreads=8)
    assert 0 < want < oracle.count(og, Motif(synth.OUT_STAR3, 3000), nthreads=8)
    assert ctx.count(dg, ctx.compile(mot)) == want
    rows = ctx.enumerate(dg, ctx.compile(mot)).cpu().numpy()
    assert (tiny.src[rows[:, 0]] == hub).all()


@pytest.mark.parametrize("tier", [0, 1])
def test_batch_mixes_labelled_and_plain(ctx, tiny_g, tiny_og, tier):
    qs = list(TINY_CASES) + [Motif(m.edges, m.delta, gap=m.gap) for m in TINY_CASES]
    old = with_params(ctx, {N.TM_PARAM_TIER: tier, N.TM_PARAM_SPLIT: 0})
    try:
        handles = [ctx.compile(m) for m in qs]
        want = [oracle.count(tiny_og, m, nthreads=8) for m in qs]
        for split in (0, 1):
            ctx.set_param(N.TM_PARAM_SPLIT, split)
            say("batch tier", tier, "split", split)
            assert ctx.count_batch(tiny_g, handles) == want
    finally:
        with_params(ctx, old)


def test_served_labelled_queries(ctx, tiny_g, tiny_og):
    srv = api.Server(ctx, tiny_g, stream_slots=2, max_batch=8, enum_pool_bytes=64 << 20, tier=1)
    try:
        for i, m in enumerate(TINY_CASES):
            srv.submit(m, enumerate=(i % 2 == 0), tag=i)
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
        if i % 2 == 0:
            assert same_rows(rows, want)


def test_labels_required_but_missing(ctx):
    g = synth.tiny_graph(0)
    dg = ctx.load_synth(g)  # no labels
    assert dg.info()["has_labels"] == 0
    with pytest.raises(N.NativeError) as ei:
        ctx.count(dg, ctx.compile(Motif(synth.TRIANGLE, 100, node_labels=[0, -1, -1])))
    assert ei.value.status == N.TM_E_INVALID
    # all free: runs
    assert ctx.count(dg, ctx.compile(Motif(synth.TRIANGLE, 10_000, node_labels=[-1, -1, -1]))) == \
        ctx.count(dg, ctx.compile(Motif(synth.TRIANGLE, 10_000)))
    with pytest.raises(N.NativeError):
        dg.set_node_labels(np.full(g.n, -1, np.int32))


# full size: the wiki-shaped graph with two random labels (as the paper's
# labelled runs use randomly generated labels)
WIKI_CASES = [
    Motif(synth.FOUR_CYCLE, 86_400, node_labels=[0, 1, 0, 1]),                     # the timed V form
    Motif(synth.FOUR_CYCLE, 86_400, gap=[21_600] * 3, node_labels=[0, 1, 0, 1]),  # the timed V+T form
    Motif(synth.FOUR_CYCLE, 86_400, gap=[21_600] * 3, anti=[(2, 0, 2, 3600)], node_labels=[0, 1, 0, 1]),  # V+T+A
    Motif(synth.OUT_STAR3, 3600, node_labels=[1, 0, 0, -1]),
]


def test_wiki_full_counts(ctx):
    say("generating wiki-shaped graph")
    g = synth.wiki_graph()
    g = synth.with_labels(g, synth.node_labels(2, g.n, 2))
    og = oracle.OracleGraph.from_graph(g)
    dg = ctx.load_synth(g)
    want = []
    for mot in WIKI_CASES:
        want.append(oracle.count(og, mot, nthreads=16))
        say("wiki labels", mot.edges, mot.node_labels, "oracle", want[-1])
        assert ctx.count(dg, ctx.compile(mot)) == want[-1]
    old = with_params(ctx, {N.TM_PARAM_TIER: 1})
    try:
        assert ctx.count_batch(dg, [ctx.compile(m) for m in WIKI_CASES]) == want
    finally:
        with_params(ctx, old)


def test_large_labels_and_int64_time_keys(ctx, tiny):
    """Label values near INT32_MAX on a graph whose time span needs 64-bit
    relative times."""
    big = (2**31 - 1) - tiny.labels.astype(np.int64) * 1_000_003
    g = synth.with_labels(synth.TemporalGraph(tiny.n, tiny.src, tiny.dst, tiny.t * 10_000, tiny.w), big)
    dg = ctx.load_synth(g)
    assert dg.info()["key_bytes"] == 8 and dg.info()["has_labels"] == 1
    og = oracle.OracleGraph.from_graph(g)
    lab = [(2**31 - 1) - v * 1_000_003 for v in (0, 1, 0, 1)]
    mot = Motif(synth.FOUR_CYCLE, 86_400 * 10_000, node_labels=lab)
    want = oracle.count(og, mot, nthreads=8)
    assert want > 0
    mm = ctx.compile(mot)
    assert ctx.count(dg, mm) == want
    assert same_rows(ctx.enumerate(dg, mm), oracle.enumerate(og, mot))
