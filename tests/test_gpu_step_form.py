"""The matchers' one-read-round loop step (TM_PARAM_STEP_FORM = 1): a step
issues the reads of every lane (search pivots, the candidate's key and
neighbour, the list offsets of a level to open) before using any, and a
binding candidate opens the next level's window in the following step. The
instances found must not change: counts, sorted instance sets and work
counters equal the oracle's for specialised and table-driven matchers, with
gaps, predicates, vertex labels, anti-edges, global-list levels, 64-bit time
keys, root ranges, splitting stress and batched launches."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from paper_2310_02800_amd import _native as N
from paper_2310_02800_amd import api, synth
from helpers import all_connected_motifs

pytestmark = pytest.mark.gpu
Motif = synth.Motif


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rows(a):
    a = a.cpu().numpy() if hasattr(a, "cpu") else np.asarray(a)
    return sorted(map(tuple, a.tolist()))


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    c.set_param(N.TM_PARAM_STEP_FORM, 1)
    assert c.get_param(N.TM_PARAM_STEP_FORM) == 1
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


def random_cases(seed, count):
    rng = np.random.Generator(np.random.PCG64(seed))
    motifs = all_connected_motifs(4, 4)
    for i in rng.choice(len(motifs), size=count, replace=False):
        me = motifs[int(i)]
        n = int(rng.integers(2, 9))
        g = synth.random_graph(rng, n, int(rng.integers(0, 60)), t_max := int(rng.integers(0, 40)))
        g = synth.with_labels(g, rng.integers(0, 2, n))
        mot = Motif(me, int(rng.integers(0, t_max + 2)))
        if len(me) > 1 and rng.random() < 0.4:
            mot.gap = [int(rng.integers(0, t_max + 1)) for _ in range(len(me) - 1)]
        if rng.random() < 0.4:
            mot.pred_edge = int(rng.integers(0, len(me)))
            mot.pred_op = int(rng.integers(0, 4))
            mot.pred_theta = float(np.float32(rng.lognormal()))
        if rng.random() < 0.3:
            mot.node_labels = [int(x) for x in rng.integers(-1, 2, mot.k)]
        if rng.random() < 0.2:
            a = int(rng.integers(0, mot.k))
            mot.anti = [(a, (a + 1) % mot.k, int(rng.integers(0, len(me))), int(rng.integers(0, 4)))]
        lo = hi = None
        if rng.random() < 0.3:
            lo = int(rng.integers(-1, t_max + 1))
            hi = int(rng.integers(lo, t_max + 2))
        yield g, mot, lo, hi


@pytest.mark.parametrize("tier", [0, 1])
def test_small_random_graphs(ctx, tier):
    """Random motif-order connected motifs (l, k <= 4) on tiny graphs with
    ties, self-loops and labels; random delta, gaps, predicates, vertex labels,
    anti-edges and root ranges."""
    old = ctx.get_param(N.TM_PARAM_TIER)
    ctx.set_param(N.TM_PARAM_TIER, tier)
    try:
        for g, mot, lo, hi in random_cases(20 + tier, 30):
            say("tier", tier, mot, lo, hi, g.m)
            og = oracle.OracleGraph.from_graph(g)
            dg = ctx.load_synth(g)
            mm = ctx.compile(mot)
            kw = {} if lo is None else dict(t_lo=lo, t_hi=hi)
            want = oracle.enumerate(og, mot, **kw)
            assert ctx.count(dg, mm, **kw) == want.shape[0]
            assert rows(ctx.enumerate(dg, mm, **kw)) == rows(want)
    finally:
        ctx.set_param(N.TM_PARAM_TIER, old)


@pytest.mark.parametrize("me", [synth.TRIANGLE, synth.FOUR_CYCLE, synth.OUT_STAR3, [(0, 1), (1, 2), (0, 2), (2, 3)],
                                [(0, 1), (1, 0), (0, 1)], [(0, 1), (2, 1), (1, 3), (3, 0), (2, 0)],
                                [(1, 0), (2, 0), (3, 0)], [(0, 1), (2, 3)]])
def test_tiny_graph_motifs(ctx, tiny_g, tiny_og, me):
    for d in (600, 10_000, 86_400):
        mot = Motif(me, d)
        say("tiny", me, d)
        mm = ctx.compile(mot)
        assert ctx.count(tiny_g, mm) == oracle.count(tiny_og, mot)
        if d == 10_000:
            assert rows(ctx.enumerate(tiny_g, mm)) == rows(oracle.enumerate(tiny_og, mot))


def test_work_counters(ctx, tiny_g, tiny_og):
    """The work-counter kernel follows the byte model (one search per window)
    in either form."""
    for mot in (synth.tiny_query(), Motif(synth.FOUR_CYCLE, 86_400, gap=[40_000] * 3)):
        c, st = oracle.count(tiny_og, mot, list_rule=1, with_stats=True)
        assert ctx.work_stats(tiny_g, ctx.compile(mot)) == st


@pytest.mark.parametrize("grid,chunk", [(1, 1), (2, 3), (4, 64)])
def test_splitting_stress(ctx, tiny_g, tiny_og, grid, chunk):
    old = {p: ctx.get_param(p) for p in (N.TM_PARAM_GRID, N.TM_PARAM_ROOT_CHUNK, N.TM_PARAM_SPLIT)}
    try:
        ctx.set_param(N.TM_PARAM_GRID, grid)
        ctx.set_param(N.TM_PARAM_ROOT_CHUNK, chunk)
        ctx.set_param(N.TM_PARAM_SPLIT, 1)
        for mot in (Motif(synth.OUT_STAR3, 60_000), Motif(synth.FOUR_CYCLE, 86_400, gap=[40_000] * 3)):
            say("split stress", grid, chunk, mot.edges)
            mm = ctx.compile(mot)
            assert ctx.count(tiny_g, mm) == oracle.count(tiny_og, mot)
            if mot.edges != synth.OUT_STAR3:
                assert rows(ctx.enumerate(tiny_g, mm)) == rows(oracle.enumerate(tiny_og, mot))
    finally:
        for p, v in old.items():
            ctx.set_param(p, v)


def test_batch_and_int64_keys(ctx, tiny, tiny_g, tiny_og):
    qs = synth.batch_queries()[:16]
    handles = [ctx.compile(m) for m in qs]
    assert ctx.count_batch(tiny_g, handles) == [oracle.count(tiny_og, m) for m in qs]
    t = tiny.t * 10_000  # span beyond int32: 64-bit relative times
    g = ctx.load_graph(tiny.n, tiny.src, tiny.dst, t, tiny.w)
    assert g.info()["key_bytes"] == 8
    og = oracle.OracleGraph(tiny.n, tiny.src, tiny.dst, t, tiny.w)
    mot = Motif(synth.FOUR_CYCLE, 3 * 10**8, gap=[10**8] * 3)
    mm = ctx.compile(mot)
    assert ctx.count(g, mm) == oracle.count(og, mot)
    assert rows(ctx.enumerate(g, mm)) == rows(oracle.enumerate(og, mot))
