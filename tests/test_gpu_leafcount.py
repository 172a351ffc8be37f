"""Closed-form counts of wide last-level windows, against the oracle.

Counting kernels count a last-level window of 32 or more candidates without
scanning it when its count has a closed form: the edges between two bound
nodes in the window, or the window's size minus the edges to each bound node
(the node itself included). This exercises every such case on a small, dense
multigraph (12 nodes, 30,000 edges, self-loops, repeated pairs and tied
times) where windows hold dozens of candidates: out- and in-stars (one new
endpoint, with self-loops to subtract), triangles and repeated pairs (both
endpoints bound), gaps, and predicates on and off the last level (a predicate
on the last level rules the closed form out), and last levels whose list and
subtracted nodes were bound before the level above (their searches are kept
across that level's iterations; with a gap before the last level only the
run starts are). Exact comparisons throughout;
the enumeration's counting pass uses the closed form and its writing pass
scans, and the library checks that they agree.
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


@pytest.fixture(scope="module")
def dense():
    return synth.random_graph(np.random.Generator(np.random.PCG64(21)), 12, 30_000, 20_000, self_loops=True)


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    c.set_param(N.TM_PARAM_LEAF_MIN, 32)  # this graph's windows hold tens of candidates
    yield c
    c.close()


@pytest.fixture(scope="module")
def dense_g(ctx, dense):
    return ctx.load_synth(dense)


@pytest.fixture(scope="module")
def dense_og(dense):
    return oracle.OracleGraph.from_graph(dense)


CASES = [
    Motif([(0, 1), (0, 2), (0, 3)], 300),                      # out-star: one new endpoint
    Motif([(1, 0), (2, 0), (3, 0)], 300),                      # in-star
    Motif([(0, 1), (1, 2), (2, 0)], 600),                      # triangle: both bound
    Motif([(0, 1), (1, 2), (2, 3), (3, 0)], 300),              # 4-cycle: both bound
    Motif([(0, 1), (1, 2)], 600),                              # 2-path: one new endpoint
    Motif([(0, 1), (1, 0)], 900),                              # reciprocal, l = 2
    Motif([(0, 1), (0, 1), (0, 1)], 900),                      # repeated pair
    Motif([(0, 1), (0, 2), (0, 3)], 600, gap=[100, 250]),      # gaps bound the window
    Motif([(0, 1), (0, 2), (2, 3)], 400, pred_edge=1, pred_op=synth.PRED_GE, pred_theta=0.8),  # predicate above
    Motif([(0, 1), (0, 2), (0, 3)], 300, pred_edge=2, pred_op=synth.PRED_LT, pred_theta=1.5),  # predicate on last
    Motif([(0, 1), (0, 2), (0, 3), (0, 4)], 150),               # 4-edge star: three fixed nodes, one new
    Motif([(1, 0), (2, 1), (3, 0)], 400),                       # last level on another list than its parent
    Motif([(1, 0), (2, 1), (3, 0)], 400, gap=[300, 120]),       # the same with a gap before the last level
]


@pytest.mark.parametrize("tier", [0, 1])
@pytest.mark.parametrize("k", range(len(CASES)))
def test_closed_form_counts(ctx, dense_g, dense_og, tier, k):
    mot = CASES[k]
    old = ctx.get_param(N.TM_PARAM_TIER)
    try:
        ctx.set_param(N.TM_PARAM_TIER, tier)
        mm = ctx.compile(mot)
        want, st = oracle.count(dense_og, mot, nthreads=8, list_rule=1, with_stats=True)
        say("case", k, "tier", tier, mot.edges, mot.delta, "count", want)
        assert ctx.count(dense_g, mm) == want
        ws = ctx.work_stats(dense_g, mm, leaf=True)
        assert {key: ws[key] for key in st} == st
        countable = mot.pred_edge != mot.l - 1
        if countable:
            assert ws["leaf_counted"] > 0  # the closed form was taken
        else:
            assert ws["leaf_counted"] == 0
        # counting pass (closed form) against the writing pass (scan): the library
        # raises if they differ; the rows themselves against the oracle when small
        lo, hi = 5_000, 5_600
        rows = ctx.enumerate(dense_g, mm, t_lo=lo, t_hi=hi)
        assert np.array_equal(sorted_rows(rows), sorted_rows(oracle.enumerate(dense_og, mot, t_lo=lo, t_hi=hi)))
        assert ctx.count(dense_g, mm, t_lo=lo, t_hi=hi) == rows.shape[0]
    finally:
        ctx.set_param(N.TM_PARAM_TIER, old)


def test_closed_form_with_splitting_and_batch(ctx, dense_g, dense_og):
    """The same counts in one batch, with splitting on and off."""
    want = [oracle.count(dense_og, m, nthreads=8) for m in CASES]
    handles = [ctx.compile(m) for m in CASES]
    old = ctx.get_param(N.TM_PARAM_SPLIT)
    try:
        for split in (0, 1):
            ctx.set_param(N.TM_PARAM_SPLIT, split)
            assert ctx.count_batch(dense_g, handles) == want
            assert [ctx.count(dense_g, h) for h in handles] == want
    finally:
        ctx.set_param(N.TM_PARAM_SPLIT, old)
