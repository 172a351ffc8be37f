"""Graph ingest on the GPU (Sec. 2.2: a time-sorted edge list with per-node
in- and out-lists; Sec. 4.2: preprocessing on the GPU), checked against numpy
on inputs large enough to exercise every level of the library's own radix
sort and prefix sums: several 8-bit digit passes, thousands of tiles, and a
degree scan over more than 4096^2 entries (three levels of tile sums).
Exact comparisons throughout."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from paper_2310_02800_amd import api, synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    yield c
    c.close()


def check_lists(g, dg):
    for direction, key, other in ((0, g.src, g.dst), (1, g.dst, g.src)):
        base = g.m if direction else 0
        want_off = base + np.concatenate(([0], np.cumsum(np.bincount(key, minlength=g.n))))
        # time order: by node, then id (ids are time order)
        off, nbr, eid, t = dg.csr(direction)
        assert np.array_equal(off.astype(np.int64), want_off)
        order = np.lexsort((np.arange(g.m), key))
        assert np.array_equal(eid, order)
        assert np.array_equal(nbr, other[order])
        assert np.array_equal(t, g.t[order] - g.t.min())
        # pair order: by node, then neighbour, then id
        off2, nbr2, eid2, t2 = dg.csr(direction + 2)
        assert np.array_equal(off2, off)
        order2 = np.lexsort((np.arange(g.m), other, key))
        assert np.array_equal(eid2, order2)
        assert np.array_equal(nbr2, other[order2])
        assert np.array_equal(t2, g.t[order2] - g.t.min())


@pytest.mark.parametrize("n,m,t_max,seed", [
    (5, 1, 10, 0),                    # one edge
    (300, 4097, 50, 1),               # one tile and a one-element tail
    (1000, 200_000, 10**6, 2),        # many tiles, heavy ties
    (20_000_000, 3_000_000, 2**40, 3),  # 25-bit node ids, three scan levels, int64 times
])
def test_ingest_matches_numpy(ctx, n, m, t_max, seed):
    say("ingest", n, m, t_max, seed)
    rng = np.random.Generator(np.random.PCG64(seed))
    g = synth.random_graph(rng, n, m, t_max)
    dg = ctx.load_synth(g)
    assert dg.info()["key_bytes"] == (8 if t_max >= 2**31 else 4)
    check_lists(g, dg)


def test_unsorted_ingest_large(ctx):
    """An input out of time order at scale: the stable time sort (64-bit keys,
    eight passes) must give time order with ties in input order."""
    rng = np.random.Generator(np.random.PCG64(11))
    n, m = 50_000, 1_000_000
    src = rng.integers(0, n, m).astype(np.int32)
    dst = ((src + 1 + rng.integers(0, n - 1, m)) % n).astype(np.int32)
    t = rng.integers(-2**40, 2**40, m).astype(np.int64)
    t[::7] = t[0]  # many ties
    dg = ctx.load_graph(n, src, dst, t)
    order = dg.edge_order()
    want = np.lexsort((np.arange(m), t))
    assert np.array_equal(order, want)
    g = synth.TemporalGraph(n=n, src=src[want], dst=dst[want], t=t[want], w=None)
    check_lists(g, dg)
