"""Compile the kernel modules of the library's standard workloads ahead of
time into the on-disk code-object cache (``_kcache/`` beside the library, or
``$TMOTIF_KERNEL_CACHE``). No device is needed: hipRTC compiles for gfx950 on
any host. A later process that needs one of these modules loads it from the
cache in milliseconds instead of compiling it.

The modules: for every motif structure of the named workloads (the small
power-law graph's triangle, the wiki-shaped graph's cycles and star and their
constrained forms, the heavy-skew motif, the 64 random batch queries), the
count, work-counter and enumeration kernels; the batched modules of the
64-query batch, of its first 16 queries and of the six wiki-shaped queries;
and the table-driven (tier 1) modules for 1-8 edges plus their batched
module. Compiles run in parallel worker processes.

    python -m paper_2310_02800_amd.prewarm [-j WORKERS]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _jobs():
    from paper_2310_02800_amd import synth
    M = synth.Motif
    singles = [synth.tiny_query(), M([(0, 1), (1, 2), (0, 2)], 5000, gap=[3000, 3000], pred_edge=1),
               synth.skew_query()]
    singles += synth.wiki_queries()
    lab = [0, 1, 0, 1]
    four = list(synth.FOUR_CYCLE)
    singles += [M(four, 86_400, node_labels=lab), M(four, 86_400, gap=[21_600] * 3, node_labels=lab),
                M(four, 86_400, gap=[21_600] * 3, anti=[(2, 0, 2, 3600)], node_labels=lab)]
    bq = synth.batch_queries()
    singles += bq
    seen = set()
    jobs = []
    for m in singles:
        key = (tuple(map(tuple, m.edges)), m.pred_edge, tuple(m.node_labels or ()), tuple(m.anti or ()))
        if key in seen:
            continue
        seen.add(key)
        jobs.append(("single", m))
    jobs += [("batch", bq, 0), ("batch", bq[:16], 0), ("batch", synth.wiki_queries(), 0)]
    jobs += [("generic", l) for l in range(0, 9)]  # 0 = the batched module of lengths 1..8
    return jobs


def _run(job):
    from paper_2310_02800_amd import api
    t0 = time.time()
    kind = job[0]
    if kind == "single":
        m = job[1]
        api.motif_compile_check(m.edges, m.delta, gap=m.gap, pred_edge=m.pred_edge, pred_op=m.pred_op,
                                pred_theta=m.pred_theta, anti=m.anti, node_labels=m.node_labels)
        what = f"motif {m.edges}"
    elif kind == "batch":
        api.batch_compile_check(job[1], tier=job[2])
        what = f"batch of {len(job[1])} (tier {job[2]})"
    else:
        api.generic_compile_check(job[1])
        what = f"table-driven l={job[1] or '1..8 batched'}"
    return what, time.time() - t0


def prewarm(workers: int | None = None, verbose: bool = True) -> int:
    """Compile every standard module not yet in the cache; returns the number
    of modules groups checked."""
    jobs = _jobs()
    workers = workers or min(8, os.cpu_count() or 1)
    t0 = time.time()
    # the heaviest (batched) compiles first so that they overlap the rest
    jobs.sort(key=lambda j: 0 if j[0] == "batch" else 1)
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        for what, dt in ex.map(_run, jobs):
            if verbose and dt > 2.0:
                print(f"prewarm: {what} compiled in {dt:.1f} s", flush=True)
    if verbose:
        print(f"prewarm: {len(jobs)} module sets ready in {time.time() - t0:.1f} s", flush=True)
    return len(jobs)


if __name__ == "__main__":
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", type=int, default=None)
    prewarm(ap.parse_args().j)
