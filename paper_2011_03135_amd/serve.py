"""Open-loop load generator for the serving runtime.

Requests arrive as a Poisson process of rate `rate` (exponential gaps from a
seeded generator); each picks a query uniformly from QUERIES and a resident
graph uniformly.  The generator submits each request at its arrival time
(never waiting for earlier ones: arrivals during busy periods queue in the
server and are admitted as slots and pool memory free up) and collects
completions as they come.  Latency = completion - arrival.
"""
import math
import time

import numpy as np

from .binding import QUERY_CLIQUE, QUERY_MOTIF, Server

QUERIES = (("TC", QUERY_CLIQUE, 3), ("4-clique", QUERY_CLIQUE, 4),
           ("3-motif", QUERY_MOTIF, 3), ("4-motif", QUERY_MOTIF, 4))


def percentile(xs, q):
    if not xs:
        return float("nan")
    xs = sorted(xs)
    i = min(len(xs) - 1, max(0, int(math.ceil(q / 100.0 * len(xs))) - 1))
    return xs[i]


def run_load(graphs, rate=500.0, n_requests=5000, n_warmup=500, seed=500, max_slots=4,
             pool_bytes=16 << 30, queries=QUERIES, server=None, progress=None, cu_percent=0):
    """Returns (stats dict, list of (graph index, query index, response)).
    `progress(done, total)` is called after every 500 completions."""
    rng = np.random.default_rng(seed)
    total = n_warmup + n_requests
    gaps = rng.exponential(1.0 / rate, size=total)
    gidx = rng.integers(0, len(graphs), size=total)
    qidx = rng.integers(0, len(queries), size=total)
    own = server is None
    srv = server or Server(max_slots=max_slots, pool_bytes=pool_bytes, cu_percent=cu_percent)
    done = {}
    t0 = Server.now() + 0.05
    arrivals = t0 + np.cumsum(gaps)
    meta = {}
    i = 0
    while i < total or srv.pending() > 0 or len(done) < total:
        now = Server.now()
        while i < total and arrivals[i] <= now:
            _, kind, k = queries[qidx[i]]
            rid = srv.submit(graphs[gidx[i]], kind, k, tag=i)
            meta[rid] = i
            i += 1
        for r in srv.poll():
            done[r.tag] = r
            if progress is not None and len(done) % 500 == 0:
                progress(len(done), total)
        if i < total:
            wait = arrivals[i] - Server.now()
            if wait > 0.0005:
                time.sleep(min(wait, 0.002))
        elif len(done) < total:
            time.sleep(0.0002)
    if own:
        srv.close()
    measured = [done[j] for j in range(n_warmup, total)]
    lat = [r.t_done - arrivals[r.tag] for r in measured]
    qwait = [r.t_admit - arrivals[r.tag] for r in measured]
    span = max(r.t_done for r in measured) - arrivals[n_warmup]
    stats = {
        "requests": n_requests, "warmup": n_warmup, "offered_rate": rate,
        "throughput_rps": n_requests / span if span > 0 else float("nan"),
        "p50_ms": 1e3 * percentile(lat, 50), "p99_ms": 1e3 * percentile(lat, 99),
        "mean_queue_ms": 1e3 * float(np.mean(qwait)),
        "failed": sum(1 for r in measured if r.status != 0),
        "max_slots": max_slots if own else None,
    }
    by_query = {}
    for j in range(n_warmup, total):
        by_query.setdefault(queries[qidx[j]][0], []).append(done[j].t_done - arrivals[j])
    stats["per_query"] = {name: {"requests": len(xs), "p50_ms": 1e3 * percentile(xs, 50),
                                 "p99_ms": 1e3 * percentile(xs, 99)}
                          for name, xs in by_query.items()}
    per = [(int(gidx[j]), int(qidx[j]), done[j]) for j in range(total)]
    return stats, per
