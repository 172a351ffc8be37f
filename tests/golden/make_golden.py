"""Write the stored expected counts of the at-scale graphs.

Calls only the CPU oracle (``oracle/``) on the seeded synthetic inputs; no
value here comes from the GPU path. Run from the repository root:

    python tests/golden/make_golden.py
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


if __name__ == "__main__":
    wiki_counts(int(os.environ.get("ORACLE_THREADS", os.cpu_count() or 1)))
