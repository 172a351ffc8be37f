"""Pins for the oracle's vertex labels (Sec. 5.4.1: a label check when a vertex
is newly matched; Table 4 row V): brute force, a partition identity, a closed
form and invariants. CPU only."""
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


def test_labels_match_brute_force_all_small_motifs():
    """Every motif-order connected motif with l <= 3, k <= 4 on tiny labelled
    graphs (3 labels) with ties and self-loops; random required labels (some
    nodes free), delta, gaps, anti-edges and root range."""
    rng = np.random.Generator(np.random.PCG64(2468))
    for mi, me in enumerate(all_connected_motifs(3, 4)):
        n = int(rng.integers(2, 6))
        m = int(rng.integers(0, 14))
        t_max = int(rng.integers(0, 10))
        g = synth.with_labels(synth.random_graph(rng, n, m, t_max), rng.integers(0, 3, n))
        k = 1 + max(max(a, b) for a, b in me)
        mot = Motif(me, int(rng.integers(0, t_max + 2)), node_labels=[int(x) for x in rng.integers(-1, 3, k)])
        if len(me) > 1 and rng.random() < 0.3:
            mot.gap = [int(rng.integers(0, t_max + 1)) for _ in range(len(me) - 1)]
        if rng.random() < 0.3:
            a = int(rng.integers(0, k))
            mot.anti = [(a, (a + 1) % k, int(rng.integers(0, len(me))), int(rng.integers(0, t_max + 2)))]
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


@pytest.fixture(scope="module")
def lab_graph():
    g = synth.tiny_graph(3, n=60, m=4000)
    return synth.with_labels(g, synth.node_labels(11, g.n, 4))


@pytest.fixture(scope="module")
def lab_og(lab_graph):
    return og_of(lab_graph)


MOTIFS = [(synth.TRIANGLE, 20_000), (synth.FOUR_CYCLE, 40_000), (synth.OUT_STAR3, 3000),
          ([(0, 1), (1, 2), (2, 3)], 10_000), ([(0, 1), (2, 3)], 200)]


@pytest.mark.parametrize("k", range(len(MOTIFS)))
def test_partition_over_one_nodes_label(lab_og, k):
    """Each match maps a motif node to exactly one labelled graph node, so the
    counts with that node's label fixed to each of the 4 labels add up to the
    unlabelled count, for every motif node; free labels (-1) change nothing."""
    me, delta = MOTIFS[k]
    nk = 1 + max(max(a, b) for a, b in me)
    base = oracle.count(lab_og, Motif(me, delta))
    assert base > 0
    assert oracle.count(lab_og, Motif(me, delta, node_labels=[-1] * nk)) == base
    for v in range(nk):
        parts = []
        for lab in range(4):
            want = [-1] * nk
            want[v] = lab
            parts.append(oracle.count(lab_og, Motif(me, delta, node_labels=want)))
        assert sum(parts) == base, (me, v, parts)


def test_closed_form_one_edge(lab_graph, lab_og):
    """One edge a->b with labels (La, Lb): the non-self-loop edges whose
    endpoints carry those labels."""
    lab = lab_graph.labels
    ok = lab_graph.src != lab_graph.dst
    for la in range(4):
        for lb in (-1, 0, 3):
            sel = ok & (lab[lab_graph.src] == la)
            if lb >= 0:
                sel &= lab[lab_graph.dst] == lb
            assert oracle.count(lab_og, Motif([(0, 1)], 0, node_labels=[la, lb])) == int(sel.sum())


def test_label_permutation_invariance(lab_graph, lab_og):
    """Renaming the labels in the graph and in the motif alike changes nothing."""
    perm = np.array([2, 0, 3, 1], np.int32)
    og2 = og_of(synth.with_labels(lab_graph, perm[lab_graph.labels]))
    for me, delta in MOTIFS[:3]:
        nk = 1 + max(max(a, b) for a, b in me)
        want = [int(x) for x in np.arange(nk) % 4]
        a = oracle.count(lab_og, Motif(me, delta, node_labels=want))
        b = oracle.count(og2, Motif(me, delta, node_labels=[int(perm[x]) for x in want]))
        assert a == b


def test_absent_label_and_missing_labels(lab_graph, lab_og):
    assert oracle.count(lab_og, Motif(synth.TRIANGLE, 20_000, node_labels=[-1, 7, -1])) == 0
    plain = og_of(synth.TemporalGraph(lab_graph.n, lab_graph.src, lab_graph.dst, lab_graph.t, lab_graph.w))
    with pytest.raises(ValueError):  # labels required, graph has none
        oracle.count(plain, Motif(synth.TRIANGLE, 20_000, node_labels=[0, -1, -1]))
    # all free: no labels needed
    assert oracle.count(plain, Motif(synth.TRIANGLE, 20_000, node_labels=[-1, -1, -1])) == \
        oracle.count(plain, Motif(synth.TRIANGLE, 20_000))
    with pytest.raises(ValueError):
        oracle.count(lab_og, Motif(synth.TRIANGLE, 20_000, node_labels=[-2, -1, -1]))
