"""Pins for the oracle's temporal anti-edges (Sec. 2.1 definition, Sec. 5.4.3
search): brute force, the walk-through's fragment (c), a closed form and
invariants. CPU only."""
from __future__ import annotations

import bisect
from collections import defaultdict

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2310_02800_amd import synth
from helpers import I64_MAX, I64_MIN, all_connected_motifs, graph_from_edges, load_golden

Motif = synth.Motif


def og_of(g):
    return oracle.OracleGraph.from_graph(g)


def rows(a):
    return sorted(map(tuple, np.asarray(a).tolist()))


def random_anti(rng, edges, t_max, n_max=2):
    """1..n_max anti-edges between motif nodes, attached to random edges, with
    windows from 0 to a little past the time range."""
    k = 1 + max(max(a, b) for a, b in edges)
    out = []
    for _ in range(int(rng.integers(1, n_max + 1))):
        a = int(rng.integers(0, k))
        b = int(rng.integers(0, k - 1))
        b = b + 1 if b >= a else b
        out.append((a, b, int(rng.integers(0, len(edges))), int(rng.integers(0, t_max + 3))))
    return out


def test_anti_edges_match_brute_force_all_small_motifs():
    """Every motif-order connected motif with l <= 3, k <= 4, each with one or
    two random anti-edges, on tiny graphs with timestamp ties, repeated pairs
    and self-loops; random delta, gaps and root range."""
    rng = np.random.Generator(np.random.PCG64(4321))
    motifs = all_connected_motifs(3, 4)
    for mi, me in enumerate(motifs):
        n = int(rng.integers(2, 5))
        m = int(rng.integers(0, 12))
        t_max = int(rng.integers(0, 10))
        g = synth.random_graph(rng, n, m, t_max)
        mot = Motif(me, int(rng.integers(0, t_max + 2)), anti=random_anti(rng, me, t_max))
        if len(me) > 1 and rng.random() < 0.3:
            mot.gap = [int(rng.integers(0, t_max + 1)) for _ in range(len(me) - 1)]
        if rng.random() < 0.3:
            t_lo = int(rng.integers(-1, t_max + 1))
            t_hi = int(rng.integers(t_lo, t_max + 2))
        else:
            t_lo, t_hi = I64_MIN, I64_MAX
        og = og_of(g)
        want = brute.enumerate_all(g, mot, t_lo, t_hi)
        assert oracle.count(og, mot, t_lo, t_hi) == len(want), (mi, mot)
        assert oracle.count(og, mot, t_lo, t_hi, list_rule=1, nthreads=2) == len(want)
        assert rows(oracle.enumerate(og, mot, t_lo, t_hi)) == want


def test_anti_edges_match_brute_force_random_seeds():
    """Random motifs of up to 4 edges whose nodes appear late (so anti-edges
    are checked below their attach level), up to 4 anti-edges."""
    rng = np.random.Generator(np.random.PCG64(77))
    for seed in range(250):
        n = int(rng.integers(2, 7))
        m = int(rng.integers(0, 12))
        t_max = int(rng.integers(0, 30))
        g = synth.random_graph(rng, n, m, t_max)
        l = int(rng.integers(1, 5))
        k = int(rng.integers(2, min(4, l + 1) + 1)) if l > 1 else 2
        me = synth.random_motif(rng, l, k) if l > 1 else [(0, 1)]
        mot = Motif(me, int(rng.integers(0, t_max + 2)), anti=random_anti(rng, me, t_max, n_max=4))
        og = og_of(g)
        want = brute.enumerate_all(g, mot)
        assert rows(oracle.enumerate(og, mot)) == want, (seed, mot)


def test_walkthrough_fragment_c():
    """Sec. 2.1, walk-through example, fragment (c), with the window's ends,
    the attached edge's own time, and an anti-edge checked below its attach
    level."""
    fx = load_golden("walkthrough_anti.json")
    g = graph_from_edges(fx["nodes"], fx["edges"])
    og = og_of(g)
    gap = [int(synth.NO_GAP) if x < 0 else x for x in fx["gap"]]
    for case in fx["cases"]:
        mot = Motif([tuple(e) for e in fx["motif"]], fx["delta"], gap=gap,
                    anti=[tuple(a) for a in case["anti"]] or None)
        got = rows(oracle.enumerate(og, mot))
        assert got == [tuple(r) for r in case["expect"]], case["why"]
        assert brute.enumerate_all(g, mot) == got


def no_reply_count(g, w):
    """Closed form of the one-edge motif a->b with the anti-edge b->a attached
    to it: the non-self-loop edges u->v with no edge v->u in [t, t + w],
    by a binary search in the sorted times of each ordered pair."""
    times = defaultdict(list)
    for s, d, t in zip(g.src.tolist(), g.dst.tolist(), g.t.tolist()):
        times[(s, d)].append(t)
    for v in times.values():
        v.sort()
    n = 0
    for s, d, t in zip(g.src.tolist(), g.dst.tolist(), g.t.tolist()):
        if s == d:
            continue
        back = times.get((d, s), [])
        i = bisect.bisect_left(back, t)
        if i == len(back) or back[i] > t + w:
            n += 1
    return n


@pytest.mark.parametrize("w", [0, 1, 7, 100, 10_000])
def test_closed_form_no_reply(w):
    g = synth.tiny_graph(5, n=30, m=3000)
    og = og_of(g)
    assert oracle.count(og, Motif([(0, 1)], 0, anti=[(1, 0, 0, w)])) == no_reply_count(g, w)


@pytest.fixture(scope="module")
def tiny():
    return synth.tiny_graph(1, n=40, m=2500)


@pytest.fixture(scope="module")
def tiny_og(tiny):
    return og_of(tiny)


ANTI_CASES = [
    (synth.TRIANGLE, 600, [(0, 2, 1, 50)]),
    ([(0, 1), (1, 2), (2, 3), (3, 0)], 900, [(2, 0, 2, 60)]),  # the paper's 4-cycle query shape
    ([(0, 1), (0, 2), (0, 3)], 500, [(1, 2, 0, 100), (3, 1, 2, 30)]),
    ([(0, 1), (1, 2)], 500, [(1, 0, 0, 40)]),
]


@pytest.mark.parametrize("k", range(len(ANTI_CASES)))
def test_anti_edges_only_remove_matches(tiny_og, k):
    """Matches with anti-edges are the matches without them minus some; a
    wider window removes at least as many; an anti-edge between nodes whose
    images are never joined in that direction removes none."""
    me, delta, anti = ANTI_CASES[k]
    base = set(rows(oracle.enumerate(tiny_og, Motif(me, delta))))
    with_anti = set(rows(oracle.enumerate(tiny_og, Motif(me, delta, anti=anti))))
    assert with_anti <= base
    wider = [(a, b, i, w * 4) for a, b, i, w in anti]
    assert set(rows(oracle.enumerate(tiny_og, Motif(me, delta, anti=wider)))) <= with_anti
    assert oracle.count(tiny_og, Motif(me, delta, anti=[(a, b, i, 0) for a, b, i, _ in anti])) >= len(with_anti)


def test_anti_edge_on_the_pair_of_its_own_edge_rules_out_everything(tiny_og):
    """Reading: every graph edge counts, so an anti-edge with the attached
    edge's own pair and direction always meets that edge at its own time."""
    assert oracle.count(tiny_og, Motif(synth.TRIANGLE, 600)) > 0
    for i, (a, b) in enumerate(synth.TRIANGLE):
        assert oracle.count(tiny_og, Motif(synth.TRIANGLE, 600, anti=[(a, b, i, 0)])) == 0


def test_anti_edge_between_unjoined_images_removes_nothing():
    """On a graph whose edges all go from even to odd nodes, an anti-edge from
    an odd image to an even one can never be met."""
    rng = np.random.Generator(np.random.PCG64(3))
    n, m = 20, 800
    src = 2 * rng.integers(0, n // 2, m)
    dst = 2 * rng.integers(0, n // 2, m) + 1
    t = rng.integers(0, 500, m)
    g = graph_from_edges(n, np.stack([src, dst, t], 1))
    og = og_of(g)
    me = [(0, 1), (2, 1)]  # 0, 2 even; 1 odd
    base = oracle.count(og, Motif(me, 200))
    assert base > 0
    assert oracle.count(og, Motif(me, 200, anti=[(1, 0, 0, 10_000), (1, 2, 1, 10_000)])) == base


def test_rejects_invalid_anti_edges():
    g = graph_from_edges(3, [(0, 1, 0), (1, 2, 1)])
    og = og_of(g)
    me = [(0, 1), (1, 2)]
    for anti in ([(0, 0, 0, 5)], [(0, 3, 0, 5)], [(0, 1, 2, 5)], [(0, 1, 0, -1)], [(0, 2, 0, 1)] * 5):
        with pytest.raises(ValueError):
            oracle.count(og, Motif(me, 10, anti=anti))


def test_huge_anti_windows_saturate():
    """A window near the int64 limit saturates instead of wrapping: the
    anti-edge then forbids the pair at any time from the attached edge on,
    which brute force (whose integers do not overflow) agrees with."""
    rng = np.random.Generator(np.random.PCG64(8))
    for seed in range(40):
        g = synth.random_graph(rng, 5, 14, 20)
        for w in (2**62, 2**63 - 1):
            mot = Motif([(0, 1), (1, 2)], 30, anti=[(2, 0, 1, w)])
            og = og_of(g)
            assert rows(oracle.enumerate(og, mot)) == brute.enumerate_all(g, mot), (seed, w)
