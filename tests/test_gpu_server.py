"""Serving loop on the GPU: every result is the same served (in a mix, with
continuous batching across stream slots) as computed alone, and equals the
oracle; enumerations are admitted by output memory. Tolerance: exact."""
from __future__ import annotations

import sys
import threading
import time

import numpy as np
import pytest

import oracle
from paper_2310_02800_amd import _native as N
from paper_2310_02800_amd import api, synth

pytestmark = pytest.mark.gpu


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


def _serve(srv, queries, gap_s, limit_s=90):
    """Submit from a thread with the given inter-arrival gaps; poll here.
    Prints progress; gives up (the test then fails) after ``limit_s``."""
    tickets = {}

    def producer():
        for i, q in enumerate(queries):
            tickets[srv.submit(q.motif, q.t_lo, q.t_hi, enumerate=q.enumerate, tag=i)] = i
            if gap_s is not None:
                time.sleep(gap_s[i])

    th = threading.Thread(target=producer)
    th.start()
    got = {}
    t0 = time.time()
    last = t0
    while len(got) < len(queries) and time.time() < t0 + limit_s:
        for r in srv.poll(64, timeout_ms=200):
            rows = srv.rows(r) if r["rows"] else None
            got[r["tag"]] = (r, rows)
            srv.release(r["ticket"])
        if time.time() - last > 10:
            last = time.time()
            say(f"served {len(got)}/{len(queries)} after {last - t0:.0f}s", srv.stats())
    th.join()
    return got


def test_served_equals_alone_and_oracle(ctx, tiny, tiny_g, tiny_og):
    # windows scaled to the tiny graph's 1e6 time span (the default delta range
    # is for a span of 2e8): 131 of the 200 counts are nonzero, none is heavy
    queries = synth.serve_queries(int(tiny.t.min()), int(tiny.t.max()), seed=7, q=200,
                                  delta_range=(300, 40_000))
    rng = np.random.Generator(np.random.PCG64(8))
    gaps = rng.exponential(0.002, len(queries))
    srv = api.Server(ctx, tiny_g, stream_slots=3, max_batch=16, enum_pool_bytes=256 << 20, tier=1)
    try:
        got = _serve(srv, queries, gaps)
        stats = srv.stats()
    finally:
        srv.stop()
    assert len(got) == len(queries)
    say("served", stats)
    assert stats["batches"] < len(queries)  # count queries were batched
    handles = {}
    old_tier = ctx.get_param(N.TM_PARAM_TIER)
    ctx.set_param(N.TM_PARAM_TIER, 1)  # alone runs use the same (precompiled) kernels
    try:
        _check(ctx, queries, got, handles, tiny_g, tiny_og)
    finally:
        ctx.set_param(N.TM_PARAM_TIER, old_tier)


def _check(ctx, queries, got, handles, tiny_g, tiny_og):
    for i, q in enumerate(queries):
        if i % 50 == 0:
            say("checking", i)
        r, rows = got[i]
        assert r["status"] == N.TM_OK, (i, r)
        want = oracle.count(tiny_og, q.motif, t_lo=q.t_lo, t_hi=q.t_hi, nthreads=4)
        assert r["count"] == want, (i, q.motif)
        key = str(q.motif)
        if key not in handles:
            handles[key] = ctx.compile(q.motif)
        assert ctx.count(tiny_g, handles[key], t_lo=q.t_lo, t_hi=q.t_hi) == want  # alone
        assert r["t_arrival_ns"] <= r["t_admit_ns"] <= r["t_launch_ns"] <= r["t_done_ns"]
        if q.enumerate:
            assert rows is not None or want == 0
            if want:
                assert np.array_equal(sorted_rows(rows),
                                      sorted_rows(oracle.enumerate(tiny_og, q.motif, t_lo=q.t_lo, t_hi=q.t_hi)))


def test_enumeration_memory_admission(ctx, tiny, tiny_g, tiny_og):
    """A pool that holds about one result at a time: enumerations wait for
    released memory and all finish; one larger than the pool reports
    TM_E_CAPACITY with its exact count."""
    mots = [synth.Motif([(0, 1), (1, 2), (0, 2)], d) for d in (20_000, 30_000, 40_000, 50_000, 60_000)]
    sizes = [oracle.count(tiny_og, m) * 3 * 8 for m in mots]
    big = synth.Motif(synth.OUT_STAR3, 86_400)
    big_rows = oracle.count(tiny_og, big)
    pool = int(max(sizes) * 1.5) + 4096
    assert big_rows * 3 * 8 > pool
    srv = api.Server(ctx, tiny_g, stream_slots=2, max_batch=4, enum_pool_bytes=pool, tier=0)
    try:
        tickets = [srv.submit(m, enumerate=True, tag=i) for i, m in enumerate(mots)]
        tb = srv.submit(big, enumerate=True, tag=99)
        done = {}
        t_end = time.time() + 90
        while len(done) < len(mots) + 1 and time.time() < t_end:
            for r in srv.poll(8, timeout_ms=200):
                rows = srv.rows(r) if r["rows"] else None
                done[r["tag"]] = (r, rows)
                srv.release(r["ticket"])
    finally:
        srv.stop()
    assert len(done) == len(mots) + 1
    for i, m in enumerate(mots):
        r, rows = done[i]
        assert r["status"] == N.TM_OK
        assert np.array_equal(sorted_rows(rows), sorted_rows(oracle.enumerate(tiny_og, m)))
    r, rows = done[99]
    assert r["status"] == N.TM_E_CAPACITY and r["count"] == big_rows and rows is None
    assert len(tickets) == 5 and tb > 0


def test_submit_rejects_bad_queries(ctx, tiny_g):
    srv = api.Server(ctx, tiny_g, stream_slots=1, max_batch=4, enum_pool_bytes=0, queue_capacity=2, tier=1)
    try:
        with pytest.raises(N.NativeError) as ei:
            srv.submit(synth.Motif([(0, 0)], 5))
        assert ei.value.status == N.TM_E_INVALID
    finally:
        srv.stop()


def test_tier2_specialises_heavy_queries(ctx):
    """Tier 2 with a probe budget of one step: count queries that do any real
    work leave their table-driven batch and run again on their own, with
    their structure's specialised kernel once it compiled (or table-driven,
    taken by an idle slot first). Every result equals the oracle's; the
    enumerations and the anti-edge query are served as under tier 1."""
    g = synth.random_graph(np.random.Generator(np.random.PCG64(77)), 3000, 400_000, 2_000_000)
    dg = ctx.load_synth(g)
    og = oracle.OracleGraph.from_graph(g)
    rng = np.random.Generator(np.random.PCG64(9))
    base = [([(0, 1), (1, 2), (2, 0)], 60_000, None), (synth.FOUR_CYCLE, 120_000, None),
            (synth.OUT_STAR3, 60_000, None), ([(0, 1), (1, 2), (2, 3)], 90_000, [30_000, 30_000])]
    qs = []
    for i in range(24):
        e, d, gap = base[i % 4]
        m = synth.Motif(list(e), int(d * rng.uniform(0.3, 1.0)), gap=gap)
        w = int(rng.uniform(0.02, 1.0) * 2_000_000)
        lo = int(rng.integers(0, 2_000_000 - w + 1))
        qs.append(synth.Query(motif=m, t_lo=lo, t_hi=lo + w, enumerate=False, arrival=0.0))
    qs.append(synth.Query(motif=synth.Motif(list(synth.FOUR_CYCLE), 60_000, anti=[(2, 0, 1, 20_000)]),
                          t_lo=0, t_hi=2_000_000, enumerate=False, arrival=0.0))
    for d in (20_000, 40_000):
        qs.append(synth.Query(motif=synth.Motif([(0, 1), (1, 2), (2, 0)], d), t_lo=500_000, t_hi=560_000,
                              enumerate=True, arrival=0.0))
    with pytest.raises(N.NativeError) as ei:
        api.Server(ctx, dg, stream_slots=1, tier=2, probe_budget=0)
    assert ei.value.status == N.TM_E_INVALID
    srv = api.Server(ctx, dg, stream_slots=3, max_batch=8, enum_pool_bytes=256 << 20, tier=2, probe_budget=1)
    try:
        got = _serve(srv, qs, None, limit_s=240)
    finally:
        srv.stop()
    assert len(got) == len(qs)
    probed = 0
    for i, q in enumerate(qs):
        r, rows = got[i]
        say("query", i, q.motif.edges, q.motif.delta, "probed", r["probed"], "tier", r["kernel_tier"])
        assert r["status"] == N.TM_OK, (i, r)
        want = oracle.count(og, q.motif, t_lo=q.t_lo, t_hi=q.t_hi, nthreads=8)
        assert r["count"] == want, (i, q.motif)
        assert r["t_arrival_ns"] <= r["t_admit_ns"] <= r["t_launch_ns"] <= r["t_done_ns"]
        if q.enumerate:
            assert not r["probed"] and r["kernel_tier"] == 1
            assert np.array_equal(sorted_rows(rows),
                                  sorted_rows(oracle.enumerate(og, q.motif, t_lo=q.t_lo, t_hi=q.t_hi)))
        elif q.motif.anti:
            assert not r["probed"] and r["kernel_tier"] == 0
        elif r["probed"]:
            probed += 1
        else:
            assert r["kernel_tier"] == 1
    say("probed", probed, "specialised", sum(1 for r, _ in got.values() if r["probed"] and r["kernel_tier"] == 0))
    assert probed > 0
    assert any(r["probed"] and r["kernel_tier"] == 0 for r, _ in got.values())


def test_tier2_stop_drains_waiting_queries(ctx, tiny_g):
    """Stopping a tier-2 server right after submission returns once every
    query has run, including those moved over the probe budget that wait for
    a compile (on the tiny graph, one structure not compiled before)."""
    srv = api.Server(ctx, tiny_g, stream_slots=2, max_batch=4, enum_pool_bytes=0, tier=2, probe_budget=1)
    mots = [synth.Motif([(0, 1), (1, 2), (2, 3), (3, 1)], d) for d in (30_000, 50_000, 70_000, 86_400)]
    mots += [synth.Motif(synth.OUT_STAR3, d) for d in (40_000, 86_400)]
    t0 = time.time()
    for i, m in enumerate(mots):
        srv.submit(m, tag=i)
    srv.stop()
    say("stopped after", time.time() - t0, "s")
