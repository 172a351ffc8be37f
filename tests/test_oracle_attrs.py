"""Pins for the oracle's general attribute constraints (Sec. 2.1: nodes and
edges may carry discrete or continuous attributes and a query may constrain
them; Sec. 5.4.1: generated checks run when a vertex or an edge is newly
matched; Sec. 6: random node and edge features): several weight predicates
(also on one edge, forming an interval), vertex label ranges and edge label
ranges. Brute force, partition identities, closed forms and invariants. CPU
only."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2310_02800_amd import synth
from helpers import I64_MAX, I64_MIN, all_connected_motifs

Motif = synth.Motif


def og_of(g):
    return oracle.OracleGraph.from_graph(g)


def rows(a):
    return sorted(map(tuple, np.asarray(a).tolist()))


def random_attrs(rng, mot, n_lab, n_elab):
    """Random constraints of every kind on a motif, each part present half of
    the time and loose enough that many cases still have matches."""
    k, l = mot.k, mot.l

    def rng_range(n_val):
        if rng.random() < 0.5:
            return -1, -1
        lo = int(rng.integers(0, n_val))
        return lo, lo + int(rng.integers(0, 2))

    if rng.random() < 0.5:
        rr = [rng_range(n_lab) for _ in range(k)]
        mot.node_labels = [a for a, _ in rr]
        if rng.random() < 0.7:
            mot.node_label_hi = [b for _, b in rr]
    if rng.random() < 0.5:
        mot.edge_labels = [rng_range(n_elab) for _ in range(l)]
    if rng.random() < 0.5:
        mot.preds = [(int(rng.integers(0, l)), int(rng.integers(0, 4)), float(np.float32(rng.lognormal(0.0, 0.5))))
                     for _ in range(int(rng.integers(1, 3)))]
    if rng.random() < 0.2:
        mot.pred_edge = int(rng.integers(0, l))
        mot.pred_op = int(rng.integers(0, 4))
        mot.pred_theta = float(np.float32(rng.lognormal(0.0, 0.5)))
    return mot


def labelled_graph(rng, n_lab, n_elab):
    n = int(rng.integers(4, 6))
    m = int(rng.integers(14, 20))
    t_max = int(rng.integers(10, 31))
    g = synth.random_graph(rng, n, m, t_max)
    return synth.with_edge_labels(synth.with_labels(g, rng.integers(0, n_lab, n)), rng.integers(0, n_elab, m)), t_max


def test_attributes_match_brute_force_all_small_motifs():
    """Every motif-order connected motif with l <= 3, k <= 4, twice, on tiny
    graphs with node labels and edge labels (2 values each), ties and
    self-loops; random label ranges, predicate sets, delta, gaps, anti-edges
    and root ranges. At least a quarter of the cases must have matches, so
    that the comparison says something."""
    rng = np.random.Generator(np.random.PCG64(97531))
    nonzero = total = 0
    for mi, me in enumerate(all_connected_motifs(3, 4) * 2):
        g, t_max = labelled_graph(rng, 2, 2)
        mot = random_attrs(rng, Motif(me, int(rng.integers(t_max // 2, t_max + 2))), 2, 2)
        if len(me) > 1 and rng.random() < 0.3:
            mot.gap = [int(rng.integers(t_max // 4, t_max + 1)) for _ in range(len(me) - 1)]
        if rng.random() < 0.2:
            a = int(rng.integers(0, mot.k))
            mot.anti = [(a, (a + 1) % mot.k, int(rng.integers(0, len(me))), int(rng.integers(0, 4)))]
        if rng.random() < 0.3:
            t_lo = int(rng.integers(-1, t_max // 2))
            t_hi = int(rng.integers(t_lo, t_max + 2))
        else:
            t_lo, t_hi = I64_MIN, I64_MAX
        og = og_of(g)
        want = brute.enumerate_all(g, mot, t_lo, t_hi)
        assert oracle.count(og, mot, t_lo, t_hi) == len(want), (mi, mot)
        assert oracle.count(og, mot, t_lo, t_hi, list_rule=1, nthreads=2) == len(want)
        assert rows(oracle.enumerate(og, mot, t_lo, t_hi)) == want
        nonzero += len(want) > 0
        total += 1
    assert nonzero >= total // 4, (nonzero, total)


def test_attributes_match_brute_force_random_4_edges():
    """120 random cases with l = 4, k <= 4 on 4-node graphs (a tenth of them
    with matches at least)."""
    rng = np.random.Generator(np.random.PCG64(8642))
    nonzero = 0
    for case in range(120):
        me = synth.random_motif(rng, 4, int(rng.integers(3, 5)))
        n, m, t_max = 4, int(rng.integers(16, 21)), int(rng.integers(20, 40))
        g = synth.random_graph(rng, n, m, t_max)
        g = synth.with_edge_labels(synth.with_labels(g, rng.integers(0, 2, n)), rng.integers(0, 2, m))
        mot = random_attrs(rng, Motif(me, t_max + 1), 2, 2)
        og = og_of(g)
        want = brute.enumerate_all(g, mot)
        assert oracle.count(og, mot) == len(want), (case, mot)
        assert rows(oracle.enumerate(og, mot)) == want
        nonzero += len(want) > 0
    assert nonzero >= 12, nonzero


@pytest.fixture(scope="module")
def attr_graph():
    g = synth.tiny_graph(4, n=60, m=4000)
    g = synth.with_labels(g, synth.node_labels(12, g.n, 5))
    return synth.with_edge_labels(g, synth.edge_labels(13, g.m, 4))


@pytest.fixture(scope="module")
def attr_og(attr_graph):
    return og_of(attr_graph)


MOTIFS = [(synth.TRIANGLE, 20_000), (synth.FOUR_CYCLE, 40_000), (synth.OUT_STAR3, 3000),
          ([(0, 1), (1, 2), (2, 3)], 10_000)]


@pytest.mark.parametrize("k", range(len(MOTIFS)))
def test_partition_over_one_edges_label(attr_og, k):
    """Each match maps a motif edge to one graph edge with one label, so the
    counts with that edge's label fixed to each of the 4 labels add up to the
    unconstrained count, for every motif edge; the full range [0, 3] and
    'any' (-1) give the unconstrained count itself."""
    me, delta = MOTIFS[k]
    base = oracle.count(attr_og, Motif(me, delta))
    assert base > 0
    assert oracle.count(attr_og, Motif(me, delta, edge_labels=[(-1, -1)] * len(me))) == base
    assert oracle.count(attr_og, Motif(me, delta, edge_labels=[(0, 3)] * len(me))) == base
    for i in range(len(me)):
        parts = []
        for lab in range(4):
            el = [(-1, -1)] * len(me)
            el[i] = (lab, lab)
            parts.append(oracle.count(attr_og, Motif(me, delta, edge_labels=el)))
        assert sum(parts) == base, (me, i, parts)


@pytest.mark.parametrize("k", range(len(MOTIFS)))
def test_label_range_is_union_of_single_labels(attr_og, k):
    """A node label range [lo, hi] admits exactly the matches of its single
    labels, so its count is their sum (same for edge label ranges)."""
    me, delta = MOTIFS[k]
    nk = 1 + max(max(a, b) for a, b in me)
    for v in range(nk):
        lo_ = [-1] * nk
        hi_ = [-1] * nk
        lo_[v], hi_[v] = 1, 3
        rng_count = oracle.count(attr_og, Motif(me, delta, node_labels=lo_, node_label_hi=hi_))
        parts = 0
        for x in (1, 2, 3):
            one = [-1] * nk
            one[v] = x
            parts += oracle.count(attr_og, Motif(me, delta, node_labels=one))
        assert rng_count == parts
    el = [(-1, -1)] * len(me)
    el[-1] = (1, 2)
    one1, one2 = list(el), list(el)
    one1[-1], one2[-1] = (1, 1), (2, 2)
    assert oracle.count(attr_og, Motif(me, delta, edge_labels=el)) == \
        oracle.count(attr_og, Motif(me, delta, edge_labels=one1)) + \
        oracle.count(attr_og, Motif(me, delta, edge_labels=one2))


def test_closed_form_one_edge(attr_graph, attr_og):
    """One edge a->b: the non-self-loop edges whose endpoint labels, edge label
    and weight satisfy the constraints, counted with numpy masks."""
    g = attr_graph
    lab, elab, w = g.labels, g.edge_labels, g.w
    ok = g.src != g.dst
    for (la, ha), (lb, hb), (le, he), preds in [
        ((0, 2), (-1, -1), (-1, -1), []),
        ((-1, -1), (3, 4), (1, 1), [(0, synth.PRED_GE, 0.5)]),
        ((1, 1), (0, 4), (0, 2), [(0, synth.PRED_GE, 0.5), (0, synth.PRED_LT, 2.0)]),
        ((-1, -1), (-1, -1), (2, 3), [(0, synth.PRED_GT, 1.0), (0, synth.PRED_LE, 1.0)]),  # empty interval
    ]:
        sel = ok.copy()
        if la >= 0:
            sel &= (lab[g.src] >= la) & (lab[g.src] <= ha)
        if lb >= 0:
            sel &= (lab[g.dst] >= lb) & (lab[g.dst] <= hb)
        if le >= 0:
            sel &= (elab >= le) & (elab <= he)
        for _, op, th in preds:
            th = np.float32(th)
            sel &= [w >= th, w > th, w <= th, w < th][op]
        mot = Motif([(0, 1)], 0, node_labels=[la, lb], node_label_hi=[ha, hb], edge_labels=[(le, he)],
                    preds=preds)
        assert oracle.count(attr_og, mot) == int(sel.sum()), (la, lb, le, preds)


def test_predicates_are_a_conjunction(attr_og):
    """Several predicates on one edge intersect: >= a and < b gives the matches
    with weight in [a, b), which with < a and >= b partition all matches."""
    me, delta = synth.FOUR_CYCLE, 40_000
    base = oracle.count(attr_og, Motif(me, delta))
    a, b = 0.6, 1.8
    for e in range(4):
        mid = oracle.count(attr_og, Motif(me, delta, preds=[(e, synth.PRED_GE, a), (e, synth.PRED_LT, b)]))
        low = oracle.count(attr_og, Motif(me, delta, preds=[(e, synth.PRED_LT, a)]))
        high = oracle.count(attr_og, Motif(me, delta, preds=[(e, synth.PRED_GE, b)]))
        assert low + mid + high == base
        # the single-predicate field and the list agree
        assert oracle.count(attr_og, Motif(me, delta, pred_edge=e, pred_op=synth.PRED_LT, pred_theta=a)) == low


def test_wider_ranges_never_lose_matches(attr_og):
    me, delta = synth.TRIANGLE, 20_000
    prev = -1
    for hi in range(0, 5):
        c = oracle.count(attr_og, Motif(me, delta, node_labels=[0, -1, -1], node_label_hi=[hi, -1, -1],
                                        edge_labels=[(-1, -1), (0, min(hi, 3)), (-1, -1)]))
        assert c >= prev
        prev = c


def test_invalid_and_missing_attributes(attr_graph, attr_og):
    g = attr_graph
    plain = og_of(synth.TemporalGraph(g.n, g.src, g.dst, g.t, g.w))
    with pytest.raises(ValueError):  # edge labels required, graph has none
        oracle.count(plain, Motif(synth.TRIANGLE, 20_000, edge_labels=[(0, 1), (-1, -1), (-1, -1)]))
    with pytest.raises(ValueError):  # empty range
        oracle.count(attr_og, Motif(synth.TRIANGLE, 20_000, node_labels=[2, -1, -1], node_label_hi=[1, -1, -1]))
    with pytest.raises(ValueError):
        oracle.count(attr_og, Motif(synth.TRIANGLE, 20_000, edge_labels=[(3, 2), (-1, -1), (-1, -1)]))
    with pytest.raises(ValueError):  # predicate on an edge the motif lacks
        oracle.count(attr_og, Motif(synth.TRIANGLE, 20_000, preds=[(3, 0, 1.0)]))
    assert oracle.count(attr_og, Motif(synth.TRIANGLE, 20_000, edge_labels=[(9, 9), (-1, -1), (-1, -1)])) == 0
