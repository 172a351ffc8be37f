"""Temporal anti-edges (Sec. 2.1, Sec. 5.4.3) on the GPU against the oracle.

Exact comparisons throughout: counts, sorted instance sets and work counters.
The cases cover an anti-edge on the root level, one checked at its attach
level, one checked below it (the attach edge's time is read back from the
root or from a kept edge id, also after the work moved to another lane or
wavefront), one on the last level (which turns the closed-form and
wavefront-cooperative last level off), a level that scans the whole edge
list, gaps and a predicate together, several anti-edges per motif, both
kinds of time key, batches that mix motifs with and without anti-edges under
both tiers, and the serving loop.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from paper_2310_02800_amd import _native as N
from paper_2310_02800_amd import api, synth
from helpers import graph_from_edges, load_golden

pytestmark = pytest.mark.gpu
Motif = synth.Motif


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def sorted_rows(a):
    a = a.cpu().numpy() if hasattr(a, "cpu") else np.asarray(a)
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a[np.lexsort(a.T[::-1])] if a.ndim == 2 and a.shape[0] else a.reshape(0, a.shape[1] if a.ndim == 2 else 0)


def same_rows(a, b):
    a, b = sorted_rows(a), sorted_rows(b)
    return a.shape[0] == b.shape[0] and (a.shape[0] == 0 or np.array_equal(a, b))


# tiny graph: 1,000 nodes, 20,000 edges over a time span of 1e6
TINY_CASES = [
    Motif([(0, 1)], 0, anti=[(1, 0, 0, 5000)]),                                 # root level, l = 1
    Motif([(0, 1), (1, 2)], 20_000, anti=[(1, 0, 0, 20_000)]),                  # root level, l = 2
    Motif(synth.TRIANGLE, 20_000, anti=[(0, 2, 1, 5000)]),                      # at its attach level
    Motif(synth.TRIANGLE, 20_000, anti=[(2, 1, 2, 20_000)]),                    # on the last level
    Motif(synth.FOUR_CYCLE, 86_400, anti=[(2, 0, 2, 20_000)]),                  # the paper's 4-cycle query shape
    Motif(synth.OUT_STAR3, 3000, anti=[(1, 2, 0, 3000), (3, 1, 1, 1000)]),      # below attach: root time, kept e1
    Motif(synth.SKEW_MOTIF, 40_000, anti=[(1, 3, 1, 20_000)]),                  # attach 1, checked at level 2
    Motif([(0, 1), (2, 3)], 200, anti=[(0, 3, 0, 300)]),                        # whole-edge-list level
    Motif([(0, 1), (1, 2), (0, 2), (2, 3)], 50_000, gap=[20_000] * 3, pred_edge=2, pred_op=synth.PRED_GE,
          pred_theta=0.5, anti=[(3, 0, 3, 10_000), (2, 1, 1, 10_000)]),         # gaps, predicate, two anti-edges
]

# dense multigraph: 12 nodes, 30,000 edges over 20,000 (windows of dozens of candidates)
DENSE_CASES = [
    Motif([(0, 1), (0, 2), (0, 3)], 300, anti=[(2, 1, 1, 50)]),    # closed-form last level stays on
    Motif([(0, 1), (0, 2), (0, 3)], 300, anti=[(3, 0, 2, 20)]),    # on the last level: closed form off
    Motif(synth.TRIANGLE, 600, anti=[(1, 0, 0, 100)]),
    Motif([(0, 1), (1, 2)], 600, anti=[(2, 0, 1, 30)]),
]


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def tiny():
    return synth.tiny_graph(0)


@pytest.fixture(scope="module")
def tiny_g(ctx, tiny):
    return ctx.load_synth(tiny)


@pytest.fixture(scope="module")
def tiny_og(tiny):
    return oracle.OracleGraph.from_graph(tiny)


@pytest.fixture(scope="module")
def dense():
    return synth.random_graph(np.random.Generator(np.random.PCG64(21)), 12, 30_000, 20_000, self_loops=True)


@pytest.fixture(scope="module")
def dense_g(ctx, dense):
    return ctx.load_synth(dense)


@pytest.fixture(scope="module")
def dense_og(dense):
    return oracle.OracleGraph.from_graph(dense)


def check_levels(mot):
    """Level at which each anti-edge is checked: its attach edge matched and
    both its nodes bound."""
    first = {}
    for j, (a, b) in enumerate(mot.edges):
        first.setdefault(a, j)
        first.setdefault(b, j)
    return [max(i, first[a], first[b]) for a, b, i, _ in mot.anti]


def with_params(ctx, values):
    """Set context parameters; returns the old values."""
    old = {p: ctx.get_param(p) for p in values}
    for p, v in values.items():
        ctx.set_param(p, v)
    return old


@pytest.mark.parametrize("tier", [0, 1])
def test_walkthrough_fragment_c(ctx, tier):
    fx = load_golden("walkthrough_anti.json")
    g = graph_from_edges(fx["nodes"], fx["edges"])
    dg = ctx.load_synth(g)
    gap = [int(synth.NO_GAP) if x < 0 else x for x in fx["gap"]]
    old = with_params(ctx, {N.TM_PARAM_TIER: tier})
    try:
        for case in fx["cases"]:
            mot = Motif([tuple(e) for e in fx["motif"]], fx["delta"], gap=gap,
                        anti=[tuple(a) for a in case["anti"]] or None)
            mm = ctx.compile(mot)
            want = np.array(case["expect"], np.int64).reshape(-1, 4)
            assert ctx.count(dg, mm) == want.shape[0], case["why"]
            assert same_rows(ctx.enumerate(dg, mm), want), case["why"]
    finally:
        with_params(ctx, old)


@pytest.mark.parametrize("split", [0, 1])
@pytest.mark.parametrize("k", range(len(TINY_CASES)))
def test_tiny_counts_rows_and_counters(ctx, tiny_g, tiny_og, k, split):
    mot = TINY_CASES[k]
    old = with_params(ctx, {N.TM_PARAM_SPLIT: split})
    try:
        mm = ctx.compile(mot)
        want, st = oracle.count(tiny_og, mot, nthreads=8, list_rule=1, with_stats=True)
        say("tiny case", k, "split", split, mot.edges, mot.anti, "count", want)
        assert ctx.count(tiny_g, mm) == want
        assert ctx.work_stats(tiny_g, mm) == st
        assert same_rows(ctx.enumerate(tiny_g, mm), oracle.enumerate(tiny_og, mot))
        lo, hi = 300_000, 420_000
        assert ctx.count(tiny_g, mm, t_lo=lo, t_hi=hi) == oracle.count(tiny_og, mot, t_lo=lo, t_hi=hi)
    finally:
        with_params(ctx, old)


@pytest.mark.parametrize("k", range(len(DENSE_CASES)))
def test_dense_wide_windows(ctx, dense_g, dense_og, k):
    mot = DENSE_CASES[k]
    old = with_params(ctx, {N.TM_PARAM_LEAF_MIN: 32})
    try:
        mm = ctx.compile(mot)
        want, st = oracle.count(dense_og, mot, nthreads=8, list_rule=1, with_stats=True)
        say("dense case", k, mot.edges, mot.anti, "count", want)
        assert ctx.count(dense_g, mm) == want
        ws = ctx.work_stats(dense_g, mm, leaf=True)
        assert {key: ws[key] for key in st} == st
        if mot.l - 1 in check_levels(mot):
            assert ws["leaf_counted"] == 0
        else:
            assert ws["leaf_counted"] > 0
        lo, hi = 5_000, 5_600
        rows = ctx.enumerate(dense_g, mm, t_lo=lo, t_hi=hi)
        assert same_rows(rows, oracle.enumerate(dense_og, mot, t_lo=lo, t_hi=hi))
        assert ctx.count(dense_g, mm, t_lo=lo, t_hi=hi) == rows.shape[0]
    finally:
        with_params(ctx, old)


@pytest.mark.parametrize("grid,chunk", [(1, 1), (2, 3), (4, 64)])
def test_splitting_stress(ctx, tiny_g, tiny_og, grid, chunk):
    """Few workgroups and tiny root chunks move most of the work between lanes
    and wavefronts, kept edge ids and bound nodes with it."""
    old = with_params(ctx, {N.TM_PARAM_GRID: grid, N.TM_PARAM_ROOT_CHUNK: chunk, N.TM_PARAM_SPLIT: 1,
                            N.TM_PARAM_SPLIT_MIN: 2})
    try:
        for k in (4, 5, 6, 8):
            mot = TINY_CASES[k]
            say("split stress", grid, chunk, mot.edges, mot.anti)
            mm = ctx.compile(mot)
            assert ctx.count(tiny_g, mm) == oracle.count(tiny_og, mot, nthreads=8)
            assert same_rows(ctx.enumerate(tiny_g, mm), oracle.enumerate(tiny_og, mot))
    finally:
        with_params(ctx, old)


@pytest.mark.parametrize("tier", [0, 1])
def test_batch_mixes_anti_and_plain_motifs(ctx, tiny_g, tiny_og, tier):
    """One launch for motifs with and without anti-edges; under the generic
    tier the plain ones share the table-driven matchers and the others get
    their own."""
    qs = list(TINY_CASES) + [Motif(m.edges, m.delta, gap=m.gap, pred_edge=m.pred_edge, pred_op=m.pred_op,
                                   pred_theta=m.pred_theta) for m in TINY_CASES]
    old = with_params(ctx, {N.TM_PARAM_TIER: tier, N.TM_PARAM_SPLIT: 0})
    try:
        handles = [ctx.compile(m) for m in qs]
        want = [oracle.count(tiny_og, m, nthreads=8) for m in qs]
        for split in (0, 1):
            ctx.set_param(N.TM_PARAM_SPLIT, split)
            say("batch tier", tier, "split", split)
            assert ctx.count_batch(tiny_g, handles) == want
        ranges = [(200_000 + 10_000 * i, 500_000 + 10_000 * i) for i in range(len(qs))]
        assert ctx.count_batch(tiny_g, handles, ranges) == [
            oracle.count(tiny_og, m, t_lo=a, t_hi=b) for m, (a, b) in zip(qs, ranges)]
    finally:
        with_params(ctx, old)


def test_int64_time_keys(ctx, tiny):
    """A time span beyond int32: the anti-edge windows scale with the times."""
    t = tiny.t * 10_000
    g = ctx.load_graph(tiny.n, tiny.src, tiny.dst, t, tiny.w)
    assert g.info()["key_bytes"] == 8
    og = oracle.OracleGraph(tiny.n, tiny.src, tiny.dst, t, tiny.w)
    for base in (TINY_CASES[4], TINY_CASES[6]):
        mot = Motif(base.edges, base.delta * 10_000, anti=[(a, b, i, w * 10_000) for a, b, i, w in base.anti])
        mm = ctx.compile(mot)
        assert ctx.count(g, mm) == oracle.count(og, mot, nthreads=8)
        assert same_rows(ctx.enumerate(g, mm), oracle.enumerate(og, mot))


def test_served_anti_queries(ctx, tiny_g, tiny_og):
    """Served counts and enumerations of anti-edge queries equal the oracle's."""
    srv = api.Server(ctx, tiny_g, stream_slots=2, max_batch=8, enum_pool_bytes=64 << 20, tier=1)
    try:
        tickets = {}
        for i, m in enumerate(TINY_CASES):
            tickets[srv.submit(m, enumerate=(i % 3 == 0), tag=i)] = i
        got = {}
        for _ in range(600):
            for r in srv.poll(64, timeout_ms=200):
                rows = srv.rows(r) if r["rows"] else None
                got[r["tag"]] = (r, rows)
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
        if i % 3 == 0 and want.shape[0]:
            assert same_rows(rows, want)


# full size: the wiki-shaped graph (1.1M nodes, 7.8M edges)
WIKI_CASES = [
    Motif(synth.FOUR_CYCLE, 86_400, gap=[21_600] * 3, anti=[(2, 0, 2, 3600)]),  # the timed T+A form
    Motif(synth.FOUR_CYCLE, 86_400, anti=[(2, 0, 2, 3600)]),
    Motif(synth.TRIANGLE, 86_400, anti=[(1, 0, 0, 3600)]),
    Motif(synth.OUT_STAR3, 3600, anti=[(1, 2, 0, 600), (3, 1, 1, 600)]),
]


@pytest.fixture(scope="module")
def wiki():
    say("generating wiki-shaped graph")
    return synth.wiki_graph()


@pytest.fixture(scope="module")
def wiki_g(ctx, wiki):
    return ctx.load_synth(wiki)


@pytest.fixture(scope="module")
def wiki_og(wiki):
    return oracle.OracleGraph.from_graph(wiki)


def test_wiki_full_counts(ctx, wiki_g, wiki_og):
    """Full-size counts, alone (autotuned launch, as timed) and in one batch,
    against the oracle's full counts."""
    want = []
    for mot in WIKI_CASES:
        want.append(oracle.count(wiki_og, mot, nthreads=16))
        say("wiki anti", mot.edges, mot.delta, mot.anti, "oracle", want[-1])
        assert ctx.count(wiki_g, ctx.compile(mot)) == want[-1]
    assert ctx.count_batch(wiki_g, [ctx.compile(m) for m in WIKI_CASES]) == want


def test_wiki_sampled_enumeration(ctx, wiki_g, wiki_og):
    """Instance sets on sampled root-time ranges of the full graph."""
    rng = np.random.Generator(np.random.PCG64(5))
    for mot in WIKI_CASES[1:3]:
        mm = ctx.compile(mot)
        for _ in range(3):
            lo = int(rng.integers(0, 190_000_000))
            hi = lo + 5_000_000
            say("wiki anti range", mot.edges, lo, hi)
            assert same_rows(ctx.enumerate(wiki_g, mm, t_lo=lo, t_hi=hi),
                             oracle.enumerate(wiki_og, mot, t_lo=lo, t_hi=hi))


def test_huge_windows_are_clamped(ctx, tiny_g, tiny_og):
    """Windows near the int64 limit (clamped to the time span on the device,
    saturated in the oracle) forbid the pair at any later time."""
    for w in (2**40, 2**63 - 1):
        mot = Motif([(0, 1), (1, 2)], 20_000, anti=[(1, 0, 0, w)])
        assert ctx.count(tiny_g, ctx.compile(mot)) == oracle.count(tiny_og, mot, nthreads=8)
