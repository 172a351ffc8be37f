"""The launch sampler (TM_PARAM_TRACE_US): samples of a running mining kernel's
control words taken from a side stream. Checks that sampling changes no
result, and that the samples are consistent: time and the chunk cursor never
go back, the last sample follows the kernel's end, and the root queue is
drained by then."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from paper_2310_02800_amd import _native as N
from paper_2310_02800_amd import api, synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    yield c
    c.close()


def check_samples(s):
    assert s.shape[0] >= 1 and s.shape[1] == 8
    assert s[-1, 6] == 1 and (s[:-1, 6] == 0).all()
    assert (np.diff(s[:, 7]) >= 0).all() and (s[:, 7] >= 0).all()  # roots handed only grow
    assert (np.diff(s[:, 0]) >= 0).all()
    assert (np.diff(s[:, 1]) >= 0).all()  # chunks taken only grow
    assert (s[:, 2] == s[0, 2]).all()
    assert s[-1, 1] >= s[-1, 2]  # queue drained at the end
    assert s[-1, 3] == 0  # no wavefront left inside a matcher
    assert (s[:, 3] >= 0).all() and (s[:, 4] >= 0).all()


def test_sampling_changes_nothing(ctx):
    g = synth.tiny_graph(0)
    dg = ctx.load_synth(g)
    og = oracle.OracleGraph.from_graph(g)
    mots = [synth.tiny_query(), synth.Motif(synth.FOUR_CYCLE, 86_400), synth.Motif(synth.OUT_STAR3, 20_000)]
    handles = [ctx.compile(m) for m in mots]
    want = [oracle.count(og, m, nthreads=8) for m in mots]
    with pytest.raises(N.NativeError):
        ctx.set_param(N.TM_PARAM_TRACE_US, 5)
    ctx.set_param(N.TM_PARAM_TRACE_US, 20)
    try:
        for split in (0, 1):
            ctx.set_param(N.TM_PARAM_SPLIT, split)
            for h, w in zip(handles, want):
                assert ctx.count(dg, h) == w
                check_samples(ctx.last_trace())
            assert ctx.count_batch(dg, handles) == want
            s = ctx.last_trace()
            check_samples(s)
            say("split", split, api.tail_summary(s))
    finally:
        ctx.set_param(N.TM_PARAM_TRACE_US, 0)
        ctx.set_param(N.TM_PARAM_SPLIT, 1)


def test_wiki_batch_samples(ctx):
    """The six headline queries as one launch: several samples while it runs,
    the queue drains before the end."""
    g = synth.wiki_graph()
    dg = ctx.load_synth(g)
    handles = [ctx.compile(m) for m in synth.wiki_queries()]
    want = ctx.count_batch(dg, handles)
    ctx.set_param(N.TM_PARAM_TRACE_US, 20)
    try:
        assert ctx.count_batch(dg, handles) == want
        s = ctx.last_trace()
    finally:
        ctx.set_param(N.TM_PARAM_TRACE_US, 0)
    check_samples(s)
    summ = api.tail_summary(s)
    say("wiki batch", summ)
    assert summ["samples"] >= 10
    assert 0 <= summ["drain_ms"] <= summ["run_ms"]
