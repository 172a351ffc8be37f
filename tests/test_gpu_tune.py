"""Autotuned launches on the GPU.

Launch settings (roots per chunk, splitting) change speed only, so every
tuned result must equal the oracle exactly: counts as integers, enumerations
as sorted instance sets. Also checks that a key is tuned once and its setting
reused (by later counts, batches and enumerations), that the tune table
survives a save / load round trip, and that the table-driven kernels with
splitting on (a setting the tuner may pick) stay exact.
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
def batch_want(tiny_og):
    return [oracle.count(tiny_og, m, nthreads=8) for m in synth.batch_queries()]


@pytest.fixture
def tuned(ctx):
    """Autotuning on with an empty table; context parameters restored after."""
    params = (N.TM_PARAM_AUTOTUNE, N.TM_PARAM_TIER, N.TM_PARAM_SPLIT)
    old = {p: ctx.get_param(p) for p in params}
    ctx.tune_clear()
    ctx.set_param(N.TM_PARAM_AUTOTUNE, 1)
    yield ctx
    for p, v in old.items():
        ctx.set_param(p, v)
    ctx.tune_clear()


def test_single_count_is_tuned_once_and_reused(tuned, tiny_g, tiny_og):
    ctx = tuned
    mot = Motif(synth.FOUR_CYCLE, 30_000, pred_edge=1, pred_op=0, pred_theta=0.5)
    mm = ctx.compile(mot)
    want = oracle.count(tiny_og, mot)
    say("tuning a 4-cycle count")
    assert ctx.count(tiny_g, mm) == want
    first = ctx.last_launch()
    assert first[2] == 1 and first[0] in (8, 16, 32, 64, 128, 256, 512, 1024, 2048) and first[1] in (0, 1)
    assert ctx.count(tiny_g, mm) == want
    assert ctx.last_launch() == first
    # an enumeration of the same key runs both passes under the tuned setting
    assert same_rows(ctx.enumerate(tiny_g, mm), oracle.enumerate(tiny_og, mot))
    assert ctx.last_launch() == first


@pytest.mark.parametrize("tier", [0, 1])
def test_tuned_batch_equals_oracle(tuned, tiny_g, batch_want, tier):
    ctx = tuned
    ctx.set_param(N.TM_PARAM_TIER, tier)
    handles = [ctx.compile(m) for m in synth.batch_queries()]
    say("tuning the 64-query batch, tier", tier)
    assert ctx.count_batch(tiny_g, handles) == batch_want
    first = ctx.last_launch()
    assert first[2] == 1
    assert ctx.count_batch(tiny_g, handles) == batch_want
    assert ctx.last_launch() == first


def test_tuned_batch_with_root_ranges(tuned, tiny_g, tiny_og):
    ctx = tuned
    ctx.set_param(N.TM_PARAM_TIER, 1)
    qs = synth.batch_queries()[:16]
    handles = [ctx.compile(m) for m in qs]
    rng = np.random.Generator(np.random.PCG64(12))
    ranges = []
    for _ in qs:
        lo = int(rng.integers(0, 900_000))
        ranges.append((lo, lo + int(rng.integers(0, 100_000))))
    want = [oracle.count(tiny_og, m, t_lo=a, t_hi=b) for m, (a, b) in zip(qs, ranges)]
    assert ctx.count_batch(tiny_g, handles, ranges) == want


def test_tune_table_round_trip(tuned, tiny_g, tiny_og, tmp_path):
    ctx = tuned
    mot = Motif(synth.OUT_STAR3, 40_000)
    mm = ctx.compile(mot)
    want = oracle.count(tiny_og, mot)
    assert ctx.count(tiny_g, mm) == want
    setting = ctx.last_launch()
    path = tmp_path / "tune.txt"
    ctx.tune_save(path)
    text = path.read_text()
    assert text.startswith("tmotif-tune 3\n")
    assert ctx.tune_clear() >= 1
    ctx.tune_load(path)
    assert ctx.count(tiny_g, mm) == want
    assert ctx.last_launch() == setting  # taken from the loaded table, no new trials
    # a version-2 table (no workgroups-per-CU column) still loads
    v2 = tmp_path / "tune2.txt"
    lines = text.splitlines()
    v2.write_text("tmotif-tune 2\n" + "".join(" ".join(l.split()[:5] + l.split()[6:]) + "\n" for l in lines[1:]))
    assert ctx.tune_clear() >= 1
    ctx.tune_load(v2)
    assert ctx.count(tiny_g, mm) == want
    assert ctx.last_launch() == setting
    bad = tmp_path / "bad.txt"
    bad.write_text("not a table\n")
    with pytest.raises(N.NativeError) as ei:
        ctx.tune_load(bad)
    assert ei.value.status == N.TM_E_INVALID


@pytest.mark.parametrize("chunk", [16, 256])
def test_generic_tier_with_splitting(ctx, tiny_g, tiny_og, chunk):
    """Table-driven kernels with splitting on: counts and enumerations exact."""
    params = (N.TM_PARAM_TIER, N.TM_PARAM_SPLIT, N.TM_PARAM_ROOT_CHUNK)
    old = {p: ctx.get_param(p) for p in params}
    try:
        ctx.set_param(N.TM_PARAM_TIER, 1)
        ctx.set_param(N.TM_PARAM_SPLIT, 1)
        ctx.set_param(N.TM_PARAM_ROOT_CHUNK, chunk)
        for mot in (Motif(synth.OUT_STAR3, 60_000), Motif(synth.FOUR_CYCLE, 86_400, gap=[40_000] * 3),
                    Motif([(0, 1), (1, 2), (0, 2), (2, 3)], 50_000, pred_edge=3, pred_op=2, pred_theta=1.2),
                    Motif([(0, 1), (2, 1), (1, 3), (3, 0), (2, 0)], 50_000, gap=[20_000] * 4)):
            say("generic split", chunk, mot.edges)
            mm = ctx.compile(mot)
            assert ctx.count(tiny_g, mm) == oracle.count(tiny_og, mot, nthreads=8)
            if mot.edges != synth.OUT_STAR3:
                assert same_rows(ctx.enumerate(tiny_g, mm), oracle.enumerate(tiny_og, mot))
    finally:
        for p, v in old.items():
            ctx.set_param(p, v)


# ---------------------------------------------------------------- work budget
HEAVY = synth.batch_queries()[36]  # ~1e9 candidate visits on the tiny graph
BUDGET = 1 << 22                   # wavefront loop steps (the heavy query needs >= 1.5e7)


@pytest.fixture
def budgeted(ctx):
    old = ctx.get_param(N.TM_PARAM_WORK_BUDGET)
    ctx.set_param(N.TM_PARAM_WORK_BUDGET, BUDGET)
    yield ctx
    ctx.set_param(N.TM_PARAM_WORK_BUDGET, old)


def test_work_budget_cancels_only_the_heavy_query(budgeted, tiny_g, tiny_og):
    ctx = budgeted
    light = [synth.tiny_query(), Motif(synth.FOUR_CYCLE, 30_000)]
    want = [oracle.count(tiny_og, m) for m in light]
    hh = ctx.compile(HEAVY)
    with pytest.raises(N.NativeError) as ei:
        ctx.count(tiny_g, hh)
    assert ei.value.status == N.TM_E_CANCELLED
    with pytest.raises(N.NativeError) as ei:
        ctx.enumerate(tiny_g, hh)
    assert ei.value.status == N.TM_E_CANCELLED
    handles = [ctx.compile(light[0]), hh, ctx.compile(light[1])]
    assert ctx.count_batch(tiny_g, handles, allow_cancel=True) == [want[0], None, want[1]]
    with pytest.raises(N.NativeError) as ei:
        ctx.count_batch(tiny_g, handles)
    assert ei.value.status == N.TM_E_CANCELLED
    for m, w in zip(light, want):  # light queries stay exact under the budget
        mm = ctx.compile(m)
        assert ctx.count(tiny_g, mm) == w
        assert same_rows(ctx.enumerate(tiny_g, mm), oracle.enumerate(tiny_og, m))


def test_work_budget_large_enough_is_exact(ctx, tiny_g, batch_want):
    old = ctx.get_param(N.TM_PARAM_WORK_BUDGET)
    try:
        ctx.set_param(N.TM_PARAM_WORK_BUDGET, 1 << 40)
        assert ctx.count(tiny_g, ctx.compile(HEAVY)) == batch_want[36]
    finally:
        ctx.set_param(N.TM_PARAM_WORK_BUDGET, old)


def test_server_cancels_over_budget_queries(ctx, tiny_g, tiny_og):
    light = [synth.tiny_query(), Motif(synth.FOUR_CYCLE, 30_000)]
    srv = api.Server(ctx, tiny_g, stream_slots=2, max_batch=8, enum_pool_bytes=64 << 20, tier=1)
    try:
        srv.submit(light[0], tag=0)
        srv.submit(HEAVY, tag=1, work_budget=BUDGET)
        srv.submit(HEAVY, tag=2, enumerate=True, work_budget=BUDGET)
        srv.submit(light[1], tag=3, enumerate=True)
        done = {}
        import time
        t_end = time.time() + 90
        while len(done) < 4 and time.time() < t_end:
            for r in srv.poll(8, timeout_ms=200):
                done[r["tag"]] = (r, srv.rows(r) if r["rows"] else None)
                srv.release(r["ticket"])
    finally:
        srv.stop()
    assert len(done) == 4
    assert done[0][0]["status"] == N.TM_OK and done[0][0]["count"] == oracle.count(tiny_og, light[0])
    assert done[1][0]["status"] == N.TM_E_CANCELLED, done[1][0]["error"]
    assert done[2][0]["status"] == N.TM_E_CANCELLED and done[2][1] is None, done[2][0]["error"]
    assert done[1][0]["error"] and done[0][0]["error"] == ""
    assert done[3][0]["status"] == N.TM_OK
    assert same_rows(done[3][1], oracle.enumerate(tiny_og, light[1]))


def test_batch_after_tuned_singles(tuned, tiny_g, batch_want):
    """Tuning some queries alone first leaves the batch exact, in the caller's
    order whatever the dispatch order."""
    ctx = tuned
    ctx.set_param(N.TM_PARAM_TIER, 1)
    qs = synth.batch_queries()
    handles = [ctx.compile(m) for m in qs]
    for i in (0, 5, 17, 36, 58):
        assert ctx.count(tiny_g, handles[i]) == batch_want[i]
    assert ctx.count_batch(tiny_g, handles) == batch_want
    rev = handles[::-1]  # results follow the caller's order whatever the dispatch order
    assert ctx.count_batch(tiny_g, rev) == batch_want[::-1]
