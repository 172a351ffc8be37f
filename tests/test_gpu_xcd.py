"""Root chunks in XCD order (TM_PARAM_XCD_ORDER = 1): each query's chunks are
contiguous root ranges in time order, cut into 8 slices, and a workgroup takes
chunks from the slice of its XCD first, then from the others. Every root must
still be searched exactly once: counts and sorted instance sets equal the
oracle's for single queries, root ranges, batches (several queries share every
XCD's chunk sequence), enumeration, splitting and root-handoff stress (few
wavefronts, so slices run dry and hand over), both matcher tiers, and a query
cancelled by its work budget inside a batch."""
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


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    c.set_param(N.TM_PARAM_XCD_ORDER, 1)
    assert c.get_param(N.TM_PARAM_XCD_ORDER) == 1
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
def wiki():
    return synth.wiki_graph(seed=5, n=20_000, m=300_000, top_degree=8000, span=2e6)


@pytest.fixture(scope="module")
def wiki_g(ctx, wiki):
    return ctx.load_synth(wiki)


@pytest.fixture(scope="module")
def wiki_og(wiki):
    return oracle.OracleGraph.from_graph(wiki)


def with_params(ctx, values):
    old = {p: ctx.get_param(p) for p in values}
    for p, v in values.items():
        ctx.set_param(p, v)
    return old


MOTIFS = [Motif(synth.TRIANGLE, 20_000), Motif(synth.FOUR_CYCLE, 20_000), Motif(synth.OUT_STAR3, 2000),
          Motif([(1, 0), (2, 0)], 5000), Motif([(0, 1), (1, 2), (2, 3)], 8000, gap=[4000, 4000])]


@pytest.mark.parametrize("tier", [0, 1])
@pytest.mark.parametrize("chunk", [1, 7, 256])
def test_counts_rows_and_batch(ctx, wiki_g, wiki_og, tier, chunk):
    old = with_params(ctx, {N.TM_PARAM_TIER: tier, N.TM_PARAM_ROOT_CHUNK: chunk, N.TM_PARAM_AUTOTUNE: 0})
    try:
        lo, hi = 900_000, 950_000
        for mot in MOTIFS:
            say("xcd tier", tier, "chunk", chunk, mot.edges, mot.delta)
            mm = ctx.compile(mot)
            want = oracle.count(wiki_og, mot, nthreads=8)
            assert ctx.count(wiki_g, mm) == want
            assert ctx.count(wiki_g, mm, t_lo=lo, t_hi=hi) == oracle.count(wiki_og, mot, t_lo=lo, t_hi=hi)
            rows = ctx.enumerate(wiki_g, mm, t_lo=lo, t_hi=hi)
            assert np.array_equal(sorted_rows(rows), sorted_rows(oracle.enumerate(wiki_og, mot, t_lo=lo, t_hi=hi)))
        handles = [ctx.compile(m) for m in MOTIFS]
        assert ctx.count_batch(wiki_g, handles) == [oracle.count(wiki_og, m, nthreads=8) for m in MOTIFS]
        rng = np.random.Generator(np.random.PCG64(9))
        ranges = []
        for _ in MOTIFS:
            a = int(rng.integers(0, 1_800_000))
            ranges.append((a, a + int(rng.integers(0, 200_000))))
        assert ctx.count_batch(wiki_g, handles, ranges) == \
            [oracle.count(wiki_og, m, t_lo=a, t_hi=b, nthreads=8) for m, (a, b) in zip(MOTIFS, ranges)]
    finally:
        with_params(ctx, old)


@pytest.mark.parametrize("grid,chunk", [(1, 64), (3, 1024), (8, 16)])
def test_split_and_handoff_stress(ctx, wiki_g, wiki_og, grid, chunk):
    """Few workgroups (some XCDs hold none, so their slices are taken by the
    others) and large or small chunks, splitting and root handoff on."""
    old = with_params(ctx, {N.TM_PARAM_SPLIT: 1, N.TM_PARAM_ROOT_HANDOFF: 1, N.TM_PARAM_GRID: grid,
                            N.TM_PARAM_ROOT_CHUNK: chunk, N.TM_PARAM_AUTOTUNE: 0})
    try:
        for mot in MOTIFS[:3]:
            say("xcd stress", grid, chunk, mot.edges)
            mm = ctx.compile(mot)
            assert ctx.count(wiki_g, mm) == oracle.count(wiki_og, mot, nthreads=8)
        handles = [ctx.compile(m) for m in MOTIFS]
        assert ctx.count_batch(wiki_g, handles) == [oracle.count(wiki_og, m, nthreads=8) for m in MOTIFS]
    finally:
        with_params(ctx, old)


def test_tiny_graph_and_64_batch(ctx, tiny_g, tiny_og):
    for me in (synth.TRIANGLE, synth.FOUR_CYCLE, synth.OUT_STAR3, [(0, 1), (2, 1), (1, 3), (3, 0), (2, 0)]):
        mot = Motif(me, 86_400)
        assert ctx.count(tiny_g, ctx.compile(mot)) == oracle.count(tiny_og, mot)
    qs = synth.batch_queries()
    handles = [ctx.compile(m) for m in qs]
    assert ctx.count_batch(tiny_g, handles) == [oracle.count(tiny_og, m) for m in qs]


def test_budget_cancels_inside_a_batch(ctx, tiny_g, tiny_og):
    heavy = synth.batch_queries()[36]  # about 1e9 candidate visits on the tiny graph
    light = [Motif(synth.TRIANGLE, 10_000), Motif(synth.FOUR_CYCLE, 20_000)]
    old = with_params(ctx, {N.TM_PARAM_WORK_BUDGET: 1 << 22, N.TM_PARAM_AUTOTUNE: 0})
    try:
        handles = [ctx.compile(m) for m in [light[0], heavy, light[1]]]
        want = [oracle.count(tiny_og, light[0]), None, oracle.count(tiny_og, light[1])]
        assert ctx.count_batch(tiny_g, handles, allow_cancel=True) == want
        with pytest.raises(N.NativeError) as ei:
            ctx.count(tiny_g, handles[1])
        assert ei.value.status == N.TM_E_CANCELLED
    finally:
        with_params(ctx, old)
