"""Write the stored expected counts of the at-scale graphs.

Calls only the CPU oracle (``oracle/``) on the seeded synthetic inputs; no
value here comes from the GPU path. Run from the repository root:

    python tests/golden/make_golden.py [wiki] [skew] [serve]
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2310_02800_amd import synth  # noqa: E402


def wiki_counts(nthreads: int):
    g = synth.wiki_graph()
    og = oracle.OracleGraph.from_graph(g)
    out = {"source": "oracle/tm_oracle.c via tests/golden/make_golden.py", "generator": synth.GEN_VERSION,
           "graph": g.name, "graph_hash": synth.content_hash(g), "queries": []}
    for mot in synth.wiki_queries():
        t0 = time.time()
        c, st = oracle.count(og, mot, nthreads=nthreads, list_rule=1, with_stats=True)
        out["queries"].append({"edges": [list(e) for e in mot.edges], "delta": mot.delta, "count": c,
                               "work": st, "oracle_s": round(time.time() - t0, 2), "threads": nthreads})
        print(mot.edges, mot.delta, c, flush=True)
    with open(os.path.join(HERE, "wiki_counts.json"), "w") as f:
        json.dump(out, f, indent=1)


def sorted_rows_sha256(rows) -> str:
    """SHA-256 of the instance set: rows as little-endian int64, in
    lexicographic order."""
    import hashlib
    import numpy as np
    a = np.ascontiguousarray(rows, dtype="<i8")
    if a.shape[0]:
        a = a[np.lexsort(a.T[::-1])]
    return hashlib.sha256(a.tobytes()).hexdigest()


def skew_counts(nthreads: int):
    """The heavy-skew graph: full count with work counters, the full instance
    set (as a hash of its sorted rows plus a few rows), and counts of a few
    root-time slices."""
    g = synth.skew_graph()
    og = oracle.OracleGraph.from_graph(g)
    mot = synth.skew_query()
    t0 = time.time()
    c, st = oracle.count(og, mot, nthreads=nthreads, list_rule=1, with_stats=True)
    count_s = time.time() - t0
    print("skew count", c, st, f"{count_s:.1f} s", flush=True)
    t0 = time.time()
    rows = oracle.enumerate(og, mot, capacity=c)
    assert rows.shape[0] == c
    import numpy as np
    # root-time slices placed by the quantiles of the instances' root times,
    # so that each holds some of them (and one before the first holds none)
    rt = np.sort(g.t[rows[:, 0]]) if c else np.array([int(g.t.min())])
    q = lambda f: int(rt[min(int(f * (rt.size - 1)), rt.size - 1)])
    slices = []
    for lo, hi in [(q(0.1), q(0.3)), (q(0.45), q(0.55)), (q(0.9), int(g.t.max())), (int(g.t.min()), q(0.0) - 1)]:
        slices.append({"t_lo": lo, "t_hi": hi, "count": oracle.count(og, mot, t_lo=lo, t_hi=hi, nthreads=nthreads)})
    srt = np.ascontiguousarray(rows, dtype=np.int64)
    srt = srt[np.lexsort(srt.T[::-1])] if srt.shape[0] else srt
    out = {"source": "oracle/tm_oracle.c via tests/golden/make_golden.py", "generator": synth.GEN_VERSION,
           "graph": g.name, "graph_hash": synth.content_hash(g),
           "motif": {"edges": [list(e) for e in mot.edges], "delta": mot.delta, "gap": list(mot.gaps())},
           "count": c, "work": st, "oracle_count_s": round(count_s, 1), "threads": nthreads,
           "rows_sha256": sorted_rows_sha256(rows), "first_rows": srt[:8].tolist(), "slices": slices}
    with open(os.path.join(HERE, "skew_counts.json"), "w") as f:
        json.dump(out, f, indent=1)


# The served stream's oracle sample: seeded choice of 200 of its 10,000
# queries; enumerations whose rows fit the test's 1 GiB row pool are stored
# as the SHA-256 of their sorted rows, larger ones by count only (the server
# returns such a query's exact count with TM_E_CAPACITY).
SERVE_SAMPLE_SEED = 5
SERVE_SAMPLE = 200
SERVE_POOL_BYTES = 1 << 30


def serve_sample_indices(n_queries: int):
    import numpy as np
    rng = np.random.Generator(np.random.PCG64(SERVE_SAMPLE_SEED))
    return sorted(int(i) for i in rng.choice(n_queries, SERVE_SAMPLE, replace=False))


def query_key(q) -> str:
    """Hash of everything that defines a served query's result."""
    import hashlib
    m = q.motif
    txt = json.dumps([[list(e) for e in m.edges], m.delta, list(m.gaps()), m.pred_edge, m.pred_op,
                      float(m.pred_theta), q.t_lo, q.t_hi, bool(q.enumerate)])
    return hashlib.sha256(txt.encode()).hexdigest()[:16]


def serve_counts(nthreads: int):
    g = synth.wiki_graph()
    og = oracle.OracleGraph.from_graph(g)
    qs = synth.serve_queries(int(g.t.min()), int(g.t.max()))
    out = {"source": "oracle/tm_oracle.c via tests/golden/make_golden.py", "generator": synth.GEN_VERSION,
           "graph": g.name, "graph_hash": synth.content_hash(g), "stream_seed": 4, "stream_queries": len(qs),
           "sample_seed": SERVE_SAMPLE_SEED, "pool_bytes": SERVE_POOL_BYTES, "queries": []}
    t_all = time.time()
    for i in serve_sample_indices(len(qs)):
        q = qs[i]
        t0 = time.time()
        c = oracle.count(og, q.motif, t_lo=q.t_lo, t_hi=q.t_hi, nthreads=nthreads)
        rec = {"index": i, "key": query_key(q), "l": q.motif.l, "enumerate": bool(q.enumerate), "count": c}
        if q.enumerate and 8 * q.motif.l * c <= SERVE_POOL_BYTES:
            rows = oracle.enumerate(og, q.motif, t_lo=q.t_lo, t_hi=q.t_hi, capacity=c)
            assert rows.shape[0] == c
            rec["rows_sha256"] = sorted_rows_sha256(rows)
        rec["oracle_s"] = round(time.time() - t0, 2)
        out["queries"].append(rec)
        print(i, q.motif.edges, q.motif.delta, q.enumerate, c, rec["oracle_s"], flush=True)
    out["oracle_total_s"] = round(time.time() - t_all, 1)
    out["threads"] = nthreads
    with open(os.path.join(HERE, "serve_sample.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    which = sys.argv[1:] or ["wiki", "skew", "serve"]
    threads = int(os.environ.get("ORACLE_THREADS", os.cpu_count() or 1))
    if "wiki" in which:
        wiki_counts(threads)
    if "skew" in which:
        skew_counts(threads)
    if "serve" in which:
        serve_counts(threads)
