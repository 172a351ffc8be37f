"""Line-sample search (TM_PARAM_LINE_SAMPLES; candidate caching, Sec. 5.1.1).

At load time the library keeps one time key per 128 bytes of the adjacency's
keys (a cache line). With the parameter on, a window opened over a list of at
least that many entries is first located among the samples inside the list,
and the search over the list then covers one line. The result must not
change: counts and sorted instance sets equal the oracle's with the search on
(several thresholds) and off, on power-law graphs (int32 keys) and on a graph
with 64-bit keys, for both matcher tiers, single and batched launches, the
one-read-round step form and splitting stress."""
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


GRAPHS = {
    "wiki": lambda: synth.wiki_graph(seed=5, n=20_000, m=300_000, top_degree=8000, span=2e6),
    "skew": lambda: synth.skew_graph(seed=6, n=50_000, m=300_000, span=3_000_000),
}
MOTIFS = {
    "wiki": [Motif(synth.TRIANGLE, 20_000), Motif(synth.FOUR_CYCLE, 20_000), Motif(synth.OUT_STAR3, 2000),
             Motif([(1, 0), (2, 0)], 5000), Motif([(0, 1), (1, 2), (2, 3)], 8000, gap=[4000, 4000]),
             Motif(synth.FOUR_CYCLE, 20_000, anti=[(2, 0, 1, 3000)])],
    "skew": [Motif(synth.TRIANGLE, 20_000), Motif(synth.FOUR_CYCLE, 20_000), Motif(synth.OUT_STAR3, 500),
             Motif([(1, 0), (2, 0)], 5000), Motif([(0, 1), (1, 2), (2, 3)], 8000, gap=[4000, 4000])],
}


@pytest.fixture(scope="module", params=list(GRAPHS))
def graph(request, ctx):
    g = GRAPHS[request.param]()
    dg = ctx.load_synth(g)
    return request.param, dg, oracle.OracleGraph.from_graph(g)


def with_params(ctx, values):
    old = {p: ctx.get_param(p) for p in values}
    for p, v in values.items():
        ctx.set_param(p, v)
    return old


@pytest.mark.parametrize("thr", [64, 1000, 0])
@pytest.mark.parametrize("tier", [0, 1])
def test_counts_and_rows(ctx, graph, thr, tier):
    name, dg, og = graph
    old = with_params(ctx, {N.TM_PARAM_LINE_SAMPLES: thr, N.TM_PARAM_TIER: tier})
    try:
        lo, hi = 900_000, 950_000
        for mot in MOTIFS[name]:
            say(name, "samples from", thr, "tier", tier, mot.edges, mot.delta, mot.gap, mot.anti)
            mm = ctx.compile(mot)
            want = oracle.count(og, mot, nthreads=8)
            assert want > 0
            assert ctx.count(dg, mm) == want
            rows = ctx.enumerate(dg, mm, t_lo=lo, t_hi=hi)
            assert np.array_equal(sorted_rows(rows), sorted_rows(oracle.enumerate(og, mot, t_lo=lo, t_hi=hi)))
        handles = [ctx.compile(m) for m in MOTIFS[name]]
        say(name, "samples from", thr, "tier", tier, "batch")
        assert ctx.count_batch(dg, handles) == [oracle.count(og, m, nthreads=8) for m in MOTIFS[name]]
    finally:
        with_params(ctx, old)


def test_with_step_form_hub_staging_and_split_stress(ctx, graph):
    name, dg, og = graph
    old = with_params(ctx, {N.TM_PARAM_LINE_SAMPLES: 64, N.TM_PARAM_STEP_FORM: 1, N.TM_PARAM_HUB_LDS: 1,
                            N.TM_PARAM_SPLIT: 1, N.TM_PARAM_GRID: 2, N.TM_PARAM_ROOT_CHUNK: 64,
                            N.TM_PARAM_AUTOTUNE: 0})
    try:
        for mot in MOTIFS[name][:3]:
            say(name, "combined", mot.edges, mot.delta)
            assert ctx.count(dg, ctx.compile(mot)) == oracle.count(og, mot, nthreads=8)
    finally:
        with_params(ctx, old)


def test_int64_keys(ctx):
    """A time span beyond int32: 64-bit keys, samples every 16 positions."""
    g = synth.wiki_graph(seed=5, n=20_000, m=300_000, top_degree=8000, span=2e6)
    t = g.t * 10_000
    dg = ctx.load_graph(g.n, g.src, g.dst, t, g.w)
    assert dg.info()["key_bytes"] == 8
    og = oracle.OracleGraph(g.n, g.src, g.dst, t, g.w)
    old = with_params(ctx, {N.TM_PARAM_LINE_SAMPLES: 64})
    try:
        for mot in (Motif(synth.TRIANGLE, 20_000 * 10_000), Motif(synth.FOUR_CYCLE, 20_000 * 10_000)):
            mm = ctx.compile(mot)
            assert ctx.count(dg, mm) == oracle.count(og, mot, nthreads=8)
            lo, hi = 900_000 * 10_000, 950_000 * 10_000
            assert np.array_equal(sorted_rows(ctx.enumerate(dg, mm, t_lo=lo, t_hi=hi)),
                                  sorted_rows(oracle.enumerate(og, mot, t_lo=lo, t_hi=hi)))
    finally:
        with_params(ctx, old)
