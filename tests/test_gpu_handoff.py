"""Tail redistribution of unstarted roots on the GPU (Sec. 5.2.2: the work
left when the queue drains is spread over idle workers). With splitting on and
TM_PARAM_ROOT_HANDOFF = 1, a wavefront whose chunk still holds 16 or more
unstarted roots once the root queue is empty hands the last half of them to
waiting wavefronts, one root per work item. Every root must still be searched
exactly once: counts and sorted instance sets equal the oracle's with the
handoff on and off, in launches shaped to leave many roots in the pools when
the queue drains (few wavefronts, large chunks), and the launch sampler shows
that roots were handed (and none with the handoff off)."""
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


# 400,000 edges: enough roots that a launch uses chunks of 256+ roots (a
# launch over R roots uses at most about R / (4 x CUs) per chunk), so a
# wavefront (64 lanes) still holds unstarted roots when the queue drains
@pytest.fixture(scope="module")
def mid():
    return synth.random_graph(np.random.Generator(np.random.PCG64(77)), 3000, 400_000, 2_000_000)


@pytest.fixture(scope="module")
def mid_g(ctx, mid):
    return ctx.load_synth(mid)


@pytest.fixture(scope="module")
def mid_og(mid):
    return oracle.OracleGraph.from_graph(mid)


MOTIFS = [Motif(synth.TRIANGLE, 60_000), Motif(synth.FOUR_CYCLE, 120_000), Motif(synth.OUT_STAR3, 60_000),
          Motif([(0, 1), (1, 2), (2, 3)], 90_000, gap=[30_000, 30_000])]


def with_params(ctx, values):
    old = {p: ctx.get_param(p) for p in values}
    for p, v in values.items():
        ctx.set_param(p, v)
    return old


@pytest.mark.parametrize("grid,chunk", [(1, 1024), (2, 256), (8, 1024), (0, 256)])
@pytest.mark.parametrize("handoff", [0, 1])
def test_counts_and_rows_with_handoff(ctx, mid_g, mid_og, grid, chunk, handoff):
    old = with_params(ctx, {N.TM_PARAM_SPLIT: 1, N.TM_PARAM_ROOT_HANDOFF: handoff, N.TM_PARAM_GRID: grid,
                            N.TM_PARAM_ROOT_CHUNK: chunk, N.TM_PARAM_AUTOTUNE: 0, N.TM_PARAM_TRACE_US: 20})
    try:
        handed = 0
        lo, hi = 500_000, 700_000
        for mot in MOTIFS:
            say("handoff", handoff, "grid", grid, "chunk", chunk, mot.edges, mot.delta)
            mm = ctx.compile(mot)
            want = oracle.count(mid_og, mot, nthreads=8)
            assert want > 0
            assert ctx.count(mid_g, mm) == want
            handed += api.tail_summary(ctx.last_trace()).get("roots_handed", 0)
            rows = ctx.enumerate(mid_g, mm, t_lo=lo, t_hi=hi)
            assert np.array_equal(sorted_rows(rows), sorted_rows(oracle.enumerate(mid_og, mot, t_lo=lo, t_hi=hi)))
        handles = [ctx.compile(m) for m in MOTIFS]
        assert ctx.count_batch(mid_g, handles) == [oracle.count(mid_og, m, nthreads=8) for m in MOTIFS]
        handed += api.tail_summary(ctx.last_trace()).get("roots_handed", 0)
        say("roots handed", handed)
        if handoff == 0:
            assert handed == 0
        elif grid in (1, 2):
            assert handed > 0  # a few wavefronts with large pools: the tail has roots to hand over
    finally:
        with_params(ctx, old)


def test_handoff_with_the_table_driven_tier(ctx, tiny_g, tiny_og):
    qs = synth.batch_queries()[:16]
    old = with_params(ctx, {N.TM_PARAM_SPLIT: 1, N.TM_PARAM_ROOT_HANDOFF: 1, N.TM_PARAM_GRID: 4,
                            N.TM_PARAM_ROOT_CHUNK: 2048, N.TM_PARAM_AUTOTUNE: 0, N.TM_PARAM_TIER: 1})
    try:
        handles = [ctx.compile(m) for m in qs]
        assert ctx.count_batch(tiny_g, handles) == [oracle.count(tiny_og, m, nthreads=8) for m in qs]
    finally:
        with_params(ctx, old)
