"""Host-side logic that needs no GPU: the load-balance summary of launch
samples, the byte models of the benchmark, and the motif descriptor's
marshalling of anti-edges and labels. CPU only."""
from __future__ import annotations

import ctypes
import importlib.util
import os

import numpy as np
import pytest

from paper_2310_02800_amd import api, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def sample(t, taken, chunks, busy, waiting=0, items=0, done=0, handed=0):
    return [t, taken, chunks, busy, waiting, items, done, handed]


def test_tail_summary_of_a_hand_made_trace():
    # queued at 0; first work seen at 1 ms; queue drained at 7 ms; kernel over by 10 ms
    s = np.array([
        sample(0, 0, 100, 0),
        sample(1_000_000, 5, 100, 64),
        sample(4_000_000, 60, 100, 64),
        sample(7_000_000, 100, 100, 40),
        sample(9_000_000, 164, 100, 10),
        sample(10_000_000, 164, 100, 0, done=1),
    ], np.int64)
    r = api.tail_summary(s)
    assert r["samples"] == 6
    assert r["run_ms"] == pytest.approx(9.0)
    assert r["drain_ms"] == pytest.approx(6.0)
    assert r["tail_ms"] == pytest.approx(3.0)
    assert r["tail_frac"] == pytest.approx(3.0 / 9.0)
    assert r["busy_after_drain_mean"] == pytest.approx((40 + 10) / 2)
    assert r["busy_peak"] == 64
    # idle share of the launch: the tail's fraction times the idle share of the peak wavefronts in it
    assert r["idle_share"] == pytest.approx(3.0 / 9.0 * (1 - 25 / 64))
    assert r["roots_handed"] == 0


def test_tail_summary_edge_cases():
    assert api.tail_summary(np.zeros((0, 8), np.int64)) == {}
    # the last sample's handed-roots column is the launch's total
    s = np.array([sample(0, 1, 10, 5), sample(5, 10, 10, 5, handed=7), sample(9, 10, 10, 0, done=1, handed=9)],
                 np.int64)
    assert api.tail_summary(s)["roots_handed"] == 9
    # never drained before the end: the tail is empty
    s = np.array([sample(0, 1, 10, 5), sample(5, 3, 10, 5), sample(9, 10, 10, 0, done=1)], np.int64)
    r = api.tail_summary(s)
    assert r["tail_ms"] == pytest.approx(0.0) and r["busy_after_drain_mean"] == 0.0


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_byte_models(bench):
    st = {"roots": 10, "windows": 4, "probes": 20, "visits": 30, "pred_visits": 2, "matches": 5,
          "leaf_counted": 1, "leaf_counted_visits": 12, "leaf_count_reads": 3}
    l = 3
    m = bench.method_bytes(st, l)
    assert m == 16 * 10 + 8 * 4 + 8 * 20 + 12 * 30 + 4 * 2 + 8 * l * 0
    # the closed form replaces the visits it did not make by the entries it read
    assert bench.algorithmic_bytes(st, l) == m - 12 * 12 + 12 * 3


def test_descriptor_marshalling():
    d, keep = api.make_desc([(0, 1), (1, 2)], 100, anti=[(2, 0, 1, 60)], node_labels=[3, -1, 0])
    assert d.n_anti == 1 and d.n_nodes == 3 and d.n_edges == 2
    anti = np.ctypeslib.as_array(ctypes.cast(d.anti, ctypes.POINTER(ctypes.c_int32)), (3,))
    win = np.ctypeslib.as_array(ctypes.cast(d.anti_delta, ctypes.POINTER(ctypes.c_int64)), (1,))
    lab = np.ctypeslib.as_array(ctypes.cast(d.node_label, ctypes.POINTER(ctypes.c_int32)), (3,))
    assert anti.tolist() == [2, 0, 1] and win.tolist() == [60] and lab.tolist() == [3, -1, 0]
    d2, _ = api.make_desc([(0, 1)], 0)
    assert d2.n_anti == 0 and not d2.anti and not d2.node_label
    with pytest.raises(ValueError):
        api.make_desc([(0, 1), (1, 2)], 100, node_labels=[0, 1])  # one per motif node
    m = synth.Motif(synth.TRIANGLE, 10, anti=[(0, 2, 1, 5)], node_labels=[0, -1, -1])
    d3, _ = api.motif_desc_of(m)
    assert d3.n_anti == 1 and d3.node_label
