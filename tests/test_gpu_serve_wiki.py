"""The served configuration at its own size on the GPU: the wiki-shaped graph
(1.1M nodes, 7.8M edges) resident in HBM and a seeded sample of 200 of the
10,000-query stream (3-6 edge motifs, delta log-uniform in [600, 86400],
root ranges of 1-100% of the span, 10% enumerations), served by the
continuous-batching server with the table-driven kernels.

Expected values come from the oracle (tests/golden/serve_sample.json, written
by tests/golden/make_golden.py, keyed by generator version, graph hash and a
hash of each query): every count, and for enumerations whose rows fit the
1 GiB row pool, the SHA-256 of the lexicographically sorted rows. Larger
enumerations return their exact count with TM_E_CAPACITY. Exact comparisons;
no work budget, so nothing is cancelled.
"""
from __future__ import annotations

import hashlib
import os
import sys
import threading
import time

import numpy as np
import pytest

from paper_2310_02800_amd import _native as N
from paper_2310_02800_amd import api, synth
from helpers import load_golden

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
from make_golden import query_key, serve_sample_indices  # noqa: E402

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def sorted_rows_sha256(rows) -> str:
    """SHA-256 of rows (device int64 [n, l]) in lexicographic order: stable
    sorts on the GPU from the last column to the first, then the bytes."""
    import torch
    r = rows
    if r.shape[0]:
        perm = torch.arange(r.shape[0], device=r.device)
        for c in range(r.shape[1] - 1, -1, -1):
            _, o = torch.sort(r[perm, c], stable=True)
            perm = perm[o]
        r = r[perm]
    a = np.ascontiguousarray(r.cpu().numpy(), dtype="<i8")
    return hashlib.sha256(a.tobytes()).hexdigest()


@pytest.fixture(scope="module")
def gold():
    return load_golden("serve_sample.json")


@pytest.fixture(scope="module")
def wiki(gold):
    say("generating the wiki-shaped graph")
    g = synth.wiki_graph()
    assert synth.content_hash(g) == gold["graph_hash"]
    assert synth.GEN_VERSION == gold["generator"]
    return g


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    yield c
    c.close()


def test_served_sample_equals_oracle(ctx, wiki, gold):
    qs = synth.serve_queries(int(wiki.t.min()), int(wiki.t.max()))
    idx = serve_sample_indices(len(qs))
    want = {r["index"]: r for r in gold["queries"]}
    assert sorted(want) == idx
    sample = [qs[i] for i in idx]
    for i, q in zip(idx, sample):
        assert query_key(q) == want[i]["key"], f"query {i} differs from the one the oracle ran"
    dg = ctx.load_synth(wiki)
    srv = api.Server(ctx, dg, stream_slots=4, max_batch=64, enum_pool_bytes=gold["pool_bytes"], tier=1)
    # arrivals: the stream's unit-rate Poisson gaps, scaled so that the
    # sample arrives over about two seconds while earlier queries still run
    arr = np.array([q.arrival for q in sample])
    gaps = np.diff(np.concatenate([[arr[0]], arr]))
    gaps = gaps * (2.0 / max(arr[-1] - arr[0], 1e-9))
    got = {}

    def producer():
        for j, q in enumerate(sample):
            time.sleep(float(gaps[j]))
            srv.submit(q.motif, q.t_lo, q.t_hi, enumerate=q.enumerate, tag=j)

    try:
        th = threading.Thread(target=producer)
        th.start()
        t0 = last = time.time()
        while len(got) < len(sample) and time.time() < t0 + 400:
            for r in srv.poll(64, timeout_ms=200):
                j = r["tag"]
                sha = None
                if r["status"] == N.TM_OK and sample[j].enumerate:
                    sha = sorted_rows_sha256(srv.rows(r))
                got[j] = (r["status"], r["count"], sha)
                srv.release(r["ticket"])
            if time.time() - last > 10:
                last = time.time()
                say(f"served {len(got)}/{len(sample)} after {last - t0:.0f} s", srv.stats())
        th.join()
    finally:
        srv.stop()
    assert len(got) == len(sample), f"only {len(got)} of {len(sample)} results"
    bad = []
    n_rows = 0
    for j, i in enumerate(idx):
        st, c, sha = got[j]
        w = want[i]
        if c != w["count"]:
            bad.append((i, "count", c, w["count"]))
            continue
        if w["enumerate"]:
            if "rows_sha256" in w:
                n_rows += 1
                if st != N.TM_OK or sha != w["rows_sha256"]:
                    bad.append((i, "rows", st))
            elif st != N.TM_E_CAPACITY:
                bad.append((i, "status", st))
        elif st != N.TM_OK:
            bad.append((i, "status", st))
    say(f"{len(sample)} served queries compared, {n_rows} enumerations by their sorted rows")
    assert not bad, bad[:10]
