"""tm_count_batch_noalloc (the batched count on the library's device scratch,
for callers that cannot allocate) against tm_count_batch, through the C ABI:
two calls in a row, the second with a smaller input, with splitting off and
on (donated work then moves through the scratch's item region), and the
errors it gives. Counts are exact; the tolerance is 0."""
from __future__ import annotations

import sys

import pytest

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


@pytest.fixture(scope="module")
def tiny_g(ctx):
    return ctx.load_synth(synth.tiny_graph(0))


@pytest.mark.parametrize("split", [0, 1])
def test_noalloc_equals_batch_twice(ctx, tiny_g, split):
    old = ctx.get_param(N.TM_PARAM_SPLIT)
    ctx.set_param(N.TM_PARAM_SPLIT, split)
    try:
        qs = synth.batch_queries()[:24]
        big = [ctx.compile(m) for m in qs]
        small = big[:6]
        t_min, t_max = 0, 1_000_000
        small_ranges = [(t_min + 1000 * i, t_max // 3 + 1000 * i) for i in range(len(small))]
        say("no-alloc: batch of", len(big), "split", split)
        want_big = ctx.count_batch(tiny_g, big)  # compiles and loads the kernels
        want_small = ctx.count_batch(tiny_g, small, ranges=small_ranges)
        got_big = ctx.count_batch_noalloc(tiny_g, big)
        assert got_big == want_big
        say("no-alloc: smaller batch")
        got_small = ctx.count_batch_noalloc(tiny_g, small, ranges=small_ranges)
        assert got_small == want_small
        # and the larger one again after the smaller one
        assert ctx.count_batch_noalloc(tiny_g, big) == want_big
    finally:
        ctx.set_param(N.TM_PARAM_SPLIT, old)


def test_noalloc_rejects_unloaded_and_oversized(ctx, tiny_g):
    fresh = [ctx.compile(synth.Motif([(0, 1), (1, 2), (2, 3), (3, 4), (4, 0)], 777))]
    with pytest.raises(N.NativeError) as ei:
        ctx.count_batch_noalloc(tiny_g, fresh)
    assert ei.value.status == N.TM_E_INVALID
    many = [ctx.compile(synth.tiny_query())] * 257
    with pytest.raises(N.NativeError) as ei:
        ctx.count_batch_noalloc(tiny_g, many)
    assert ei.value.status == N.TM_E_INVALID
    assert "256" in str(ei.value)
