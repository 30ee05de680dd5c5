#!/usr/bin/env python3
"""Throughput of the pattern-mining hot path on one MI355X.

Workload of one step: an RMAT graph of scale 20 (2^20 vertices, exactly
16 * 2^20 distinct undirected edges, a, b, c, d = 0.57, 0.19, 0.19, 0.05,
seed 20, ids permuted) given as its raw edge stream (17,978,493 entries with
repeats and self-loops) resident in HBM.  A step builds the canonical CSR and
the degree-ordered DAG on the device and counts triangles, 4-cliques and
5-cliques in one local-graph pass (gpm_clique_counts); the per-size calls
(gpm_count) are timed separately.  Inputs are synthetic and seeded.

One JSON line:
  value             undirected edges per second of the whole step
  matches_per_sec   (triangles + 4-cliques + 5-cliques) per second
  per_problem       each per-size counting call timed alone (HIP events
                    around it on the launch stream): ms, edges/s, matches/s
  phases_ms         per-kernel milliseconds per step, HIP events recorded on
                    the launch stream by the library's timing spans
  roofline          the dominant kernel against its bound
  phase_rooflines   the triangle and 4-clique calls against the HBM roofline
                    on the algorithmic bytes of their pair scans
  batched_vs_plain  20,000 random geometric graphs (n in [10, 200]), induced
                    4-motif counts: one fused launch replayed from a HIP
                    graph (configuration picked by the autotuner) vs one
                    library call per graph on prebuilt graphs
  serving           Poisson load of mixed queries on 8 resident graphs:
                    throughput and p50/p99 latency
  cpu_baseline      the CPU oracle on a bounded sample of the same workload
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


HBM_PEAK_GBS = 8000.0
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz: one 32-bit integer VALU op per lane
# per clock (a wave64 instruction occupies a 16-lane SIMD for 4 clocks)
INT32_VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# algorithmic int32 ops per local triangle of the 5-clique kernel: the AND and
# the population count of one 64-bit candidate word (2 + 2 32-bit ops)
OPS_PER_LOCAL_TRIANGLE = 4


# Bytes beyond L2 per launch of the dominant kernel from two rocprofv3 counter
# runs: TCC EA read requests x 128 B (32 B for TCC_EA0_RDREQ_32B) and write
# requests x 64 B (TCC_EA0_WRREQ_64B) or 32 B
# (profiles/rmat20_cliques_hbm_traffic.md); valid only while the kernel's
# source is the one measured.
MEASURED_TRAFFIC = {
    "kernel": "k_lg5<1024>",
    "source": "paper_2011_03135_amd/csrc/local_graph.hip",
    "source_sha256_prefix": "0929cc93784b2dcc",
    "lg5_slice": 1 << 20,   # the task size the counters were taken at
    "bytes_read": 4307177 * 128,
    "bytes_written": 30690 * 32,
}


def measured_traffic(kernel, lg5_slice):
    import hashlib
    t = MEASURED_TRAFFIC
    if kernel != t["kernel"] or lg5_slice != t["lg5_slice"]:
        return None
    with open(os.path.join(ROOT, t["source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest()[:16] != t["source_sha256_prefix"]:
            return None
    return t["bytes_read"] + t["bytes_written"]


def dag_class_bytes(off, adj, dmin, dmax, kmin):
    """Algorithmic bytes of one triangle/local-graph-build launch over the
    roots u with dmin < d+(u) <= dmax and d+(u) >= kmin: per root, its
    out-list (4 B per arc); per out-neighbour v, v's two offsets (8 B) and
    v's out-list (4 B per entry, the (v, w) pairs)."""
    n = off.shape[0] - 1
    deg = np.diff(off).astype(np.int64)
    rows = np.repeat(np.arange(n, dtype=np.int64), deg)
    cols = adj.astype(np.int64)
    fwd = (deg[rows] < deg[cols]) | ((deg[rows] == deg[cols]) & (rows < cols))
    src, dst = rows[fwd], cols[fwd]
    dout = np.bincount(src, minlength=n)
    pairs_root = np.bincount(src, weights=dout[dst], minlength=n).astype(np.int64)
    sel = (dout > dmin) & (dout <= dmax) & (dout >= kmin) & (pairs_root > 0)
    arcs = int(dout[sel].sum())
    pairs = int(pairs_root[sel].sum())
    return 12 * arcs + 4 * pairs, arcs, pairs


def roofline(dom, ms, units, off, adj, lg5_slice):
    if dom.startswith("k_lg5"):
        ops = OPS_PER_LOCAL_TRIANGLE * units
        ach = ops / (ms * 1e-3) / 1e12
        return {"kernel": dom, "bound": "alu", "achieved": ach, "peak": INT32_VALU_PEAK_TOPS,
                "unit": "TOP/s (int32)", "frac": ach / INT32_VALU_PEAK_TOPS,
                "traffic": measured_traffic(dom, lg5_slice), "traffic_unit": "bytes per launch",
                "units_per_launch": units, "unit_name": "local triangles",
                "ops_per_unit": OPS_PER_LOCAL_TRIANGLE, "avg_launch_ms": ms}
    if dom.startswith("k_tc_flat"):
        dmin, dmax, kmin = (0, 256, 2) if "<256" in dom else (256, 1024, 2)
    elif dom.startswith("k_clique_wave"):
        dmin, dmax, kmin = 0, 64, int(dom.split("<")[1][0]) - 1
    elif "<256>" in dom or "<256," in dom:
        dmin, dmax, kmin = 64, 256, 3
    else:
        dmin, dmax, kmin = 256, 1024, 3
    b, arcs, pairs = dag_class_bytes(off, adj, dmin, dmax, kmin)
    ach = b / (ms * 1e-3) / 1e9
    return {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": None, "alg_bytes_per_launch": b,
            "pairs_per_launch": pairs, "device_units": units, "avg_launch_ms": ms}


def phase_roofline(name, ms, off, adj, kmin):
    """HBM roofline of a whole counting call (all its kernels) on the
    algorithmic bytes of its pair scan: every root with d+ >= kmin reads its
    out-list and its out-neighbours' offsets (12 B per arc) and each
    out-neighbour's out-list once (4 B per pair); everything after that runs
    on chip (LDS hash, LDS bit rows)."""
    b, arcs, pairs = dag_class_bytes(off, adj, 0, 1 << 30, kmin)
    ach = b / (ms * 1e-3) / 1e9
    return {"phase": name, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "alg_bytes": b, "arcs": arcs, "pairs": pairs, "ms": ms}


def cpu_baseline(e, stride, ks, threads, gpu_counts):
    """The oracle (unchanged) on a bounded share of the step's work: its
    core-ordered DAG is built first, outside the timed region (the paper
    times mining, not preprocessing), then the k-cliques rooted at every
    `stride`-th vertex of the core order are counted for every k of the
    step.  The rate is the whole graph's edges over the share's time scaled
    by the stride; clique_share says how much of the step's output the share
    covered."""
    import oracle
    off, adj = oracle.canonical_csr(e.n, e.u, e.v)
    m = adj.shape[0] // 2
    t0 = time.perf_counter()
    dag = oracle.CoreDag(off, adj)
    prep = time.perf_counter() - t0
    t0 = time.perf_counter()
    sampled = [dag.clique_count_sampled(k, stride, 0, threads) for k in ks]
    dt = time.perf_counter() - t0
    dag.close()
    return {
        "value": m / (dt * stride),
        "unit": "edges/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"cliques k={list(ks)} rooted at every {stride}-th vertex of the core order "
                  f"of the same rmat graph ({dt:.1f} s, DAG prebuilt in {prep:.1f} s outside "
                  f"the timing); rate = m / (time * {stride})",
        "sampled_counts": sampled,
        "clique_share": sum(sampled) / max(1, sum(gpu_counts)),
    }


def batch_leg(gpm, torch, G, plain_graphs, replays):
    """20,000 random geometric graphs, induced 4-motif counts.  Batched: one
    fused persistent launch per tier (configuration picked by the
    autotuner) replayed from a HIP graph.  Plain, same kernels: one
    gpm_batch_motif_count call per graph (G = 1, the graph's own vertex
    range of the same union graph), stream-serialised, no capture.  Plain,
    general call: gpm_motif_count on each graph built on its own, timed on
    `plain_graphs` graphs and scaled to all."""
    import ctypes
    import graphgen
    dev = torch.device("cuda:0")
    batch = graphgen.rgg_batch(G, seed=2020)
    u = torch.from_numpy(batch.u).to(dev)
    v = torch.from_numpy(batch.v).to(dev)
    g = gpm.Graph.build(batch.n, u, v)
    voff = torch.from_numpy(batch.voff.astype(np.int32)).to(dev)
    ws = torch.empty(gpm.binding.batch_workspace_bytes(G, 4), dtype=torch.uint8, device=dev)
    out = torch.zeros((G, 7), dtype=torch.int64, device=dev)
    # the autotuner picks team width, tiers and teams per CU on this batch
    cfg, tuned_ms, _ = gpm.batch_autotune(g, voff, 4, reps=3, ws=ws, out=out)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        gpm.batch_motif_count(g, voff, 4, ws=ws, out=out, config=cfg)
    torch.cuda.current_stream().wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        gpm.batch_motif_count(g, voff, 4, ws=ws, out=out, config=cfg)
    graph.replay()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(replays):
        graph.replay()
    b.record()
    torch.cuda.synchronize()
    batched_ms = a.elapsed_time(b) / replays
    batched = out.cpu().numpy()

    # plain, same kernels: G calls with G = 1 on the graph's offset pair
    lib = gpm.binding.load()
    ws1 = torch.empty(gpm.binding.batch_workspace_bytes(1, 4), dtype=torch.uint8, device=dev)
    out1 = torch.zeros((G, 7), dtype=torch.int64, device=dev)
    cfgp = ctypes.byref(cfg)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    gh, wsp, wsn = g.handle, ctypes.c_void_p(ws1.data_ptr()), ws1.numel()
    vp = [ctypes.c_void_p(voff.data_ptr() + 4 * i) for i in range(G)]
    op = [ctypes.c_void_p(out1.data_ptr() + 56 * i) for i in range(G)]

    def plain_loop():
        for i in range(G):
            rc = lib.gpm_batch_motif_count_config(gh, vp[i], 1, 4, cfgp, wsp, wsn, op[i], st)
            if rc:
                raise RuntimeError(f"gpm_batch_motif_count_config failed: {rc}")

    plain_loop()   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    a.record()
    plain_loop()
    b.record()
    torch.cuda.synchronize()
    plain_same_ms = a.elapsed_time(b)
    plain_same_wall_ms = (time.perf_counter() - t0) * 1e3
    same_kernels_equal = bool(np.array_equal(out1.cpu().numpy(), batched))

    # plain, general call: one gpm_motif_count per separately built graph
    P = min(plain_graphs, G)
    graphs = []
    for i in range(P):
        e = batch.graph(i)
        graphs.append(gpm.Graph.build(e.n, torch.from_numpy(e.u).to(dev),
                                      torch.from_numpy(e.v).to(dev)))
    wsb = max(gpm.binding.motif_workspace_bytes(gi, 4) for gi in graphs)
    pws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    pout = torch.zeros((P, 7), dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    a.record()
    for i, gi in enumerate(graphs):
        gpm.motif_count(gi, 4, ws=pws, out=pout[i])
    b.record()
    torch.cuda.synchronize()
    plain_ms = a.elapsed_time(b)
    same = bool(np.array_equal(pout.cpu().numpy()[:, :6], batched[:P, :6]))
    plain_equiv = plain_ms * G / P
    return {
        "workload": f"rgg batch G={G} (n uniform in [10, 200], seed 2020), induced 4-motifs",
        "batched_ms": batched_ms,
        "autotuned_config": cfg.as_dict(), "autotune_ms": tuned_ms,
        "graphs_per_sec_batched": G / (batched_ms * 1e-3),
        "plain_same_kernels": {
            "what": "one gpm_batch_motif_count call per graph (G = 1), same configuration, "
                    "stream-serialised, no graph capture",
            "ms": plain_same_ms, "host_wall_ms": plain_same_wall_ms,
            "graphs_per_sec": G / (plain_same_ms * 1e-3),
            "equals_batched": same_kernels_equal},
        "speedup": plain_same_ms / batched_ms,
        "plain_general_call": {
            "what": "one gpm_motif_count call per separately built graph (the general "
                    "local-count pipeline, dozens of launches per graph)",
            "ms_measured": plain_ms, "graphs_measured": P, "ms_for_all": plain_equiv,
            "speedup_vs_batched": plain_equiv / batched_ms,
            "equals_batched": same},
        "batched_status_ok": bool((batched[:, 6] == 0).all()),
    }


def device_concurrency(resps):
    """Mean number of requests in flight on the device: the sum of the
    requests' device spans (events on their slot streams before and after
    their work) over the span from the first start to the last end."""
    spans = [(r.d_start, r.d_end) for r in resps if r.d_start >= 0.0]
    if not spans:
        return None
    busy = sum(b - a for a, b in spans)
    total = max(b for _, b in spans) - min(a for a, _ in spans)
    return busy / total if total > 0 else None


def serve_compare(gpm, torch, graphs, n_requests=1000, seed=502):
    """The same seeded request list (query and graph drawn uniformly) run
    plain (one synchronous library call after another on one stream, as a
    client without the server would) and through the server, all requests
    submitted at once (a saturating load), with one slot and with four.
    Throughput = requests / wall time; latency = submission to result on
    the host."""
    from paper_2011_03135_amd.binding import QUERY_CLIQUE, Server
    from paper_2011_03135_amd.serve import QUERIES, percentile
    rng = np.random.default_rng(seed)
    gi = rng.integers(0, len(graphs), size=n_requests)
    qi = rng.integers(0, len(QUERIES), size=n_requests)

    def plain_call(g, q):
        _, kind, k = QUERIES[q]
        if kind == QUERY_CLIQUE:
            return [gpm.count(g, gpm.clique(k))]
        return gpm.motif_count(g, k)

    for g in graphs:                      # warm-up: every query on every graph once
        for q in range(len(QUERIES)):
            plain_call(g, q)
    torch.cuda.synchronize()
    lat, plain_res = [], []
    t0 = time.perf_counter()
    for j in range(n_requests):
        ts = time.perf_counter()
        plain_res.append(plain_call(graphs[gi[j]], qi[j]))
        lat.append(time.perf_counter() - ts)
    t_plain = time.perf_counter() - t0
    res = {"requests": n_requests, "seed": seed,
           "plain": {"throughput_rps": n_requests / t_plain, "wall_s": t_plain,
                     "p50_ms": 1e3 * percentile(lat, 50), "p99_ms": 1e3 * percentile(lat, 99)}}

    def served(slots, cu_percent):
        srv = Server(max_slots=slots, pool_bytes=48 << 30, cu_percent=cu_percent)
        t0 = Server.now()
        for j in range(n_requests):
            _, kind, k = QUERIES[qi[j]]
            srv.submit(graphs[gi[j]], kind, k, tag=j)
        done = {}
        while len(done) < n_requests:
            for r in srv.poll():
                done[r.tag] = r
            time.sleep(0.0002)
        srv.close()
        rs = [done[j] for j in range(n_requests)]
        wall = max(r.t_done for r in rs) - t0
        lat = [r.t_done - r.t_submit for r in rs]
        return {"slots": slots, "cu_percent": cu_percent,
                "throughput_rps": n_requests / wall, "wall_s": wall,
                "p50_ms": 1e3 * percentile(lat, 50), "p99_ms": 1e3 * percentile(lat, 99),
                "device_requests_in_flight": device_concurrency(rs),
                "failed": sum(1 for r in rs if r.status != 0),
                "equals_plain": all(rs[j].counts() == plain_res[j] for j in range(n_requests))}

    for slots, pct in ((1, 100), (4, 50), (4, 100)):
        key = f"server_{slots}slot" + ("" if slots == 1 else f"_cu{pct}")
        res[key] = served(slots, pct)
        res[key]["vs_plain"] = res[key]["throughput_rps"] / res["plain"]["throughput_rps"]
    return res


def serve_leg(gpm, torch, g20, scale, requests, warmup):
    """Open-loop serving load: Poisson arrivals at 500 requests/s, each a
    query drawn uniformly from {TC, 4-clique, 3-motif, 4-motif} on one of 8
    resident graphs drawn uniformly (RMAT scales 12..18 and the step's
    scale-20 graph, each tuned once at load).  Every request recomputes its
    answer.  Then the same kind of mix saturating the server, against plain
    back-to-back calls on the same graphs."""
    import graphgen
    from paper_2011_03135_amd.serve import run_load
    dev = torch.device("cuda:0")
    graphs, names = [], []
    for s in (12, 13, 14, 15, 16, 17, 18):
        e = graphgen.rmat(s, seed=s if s == 18 else 1000 + s)
        graphs.append(gpm.Graph.build(e.n, torch.from_numpy(e.u).to(dev),
                                      torch.from_numpy(e.v).to(dev)))
        names.append(f"rmat{s}")
    graphs.append(g20)
    names.append(f"rmat{scale}")
    # each resident graph's task granularity is tuned once when it is
    # loaded (set-up, untimed; the step's graph already is)
    for g in graphs[:-1]:
        g.autotune()
    torch.cuda.synchronize()
    stats, per = run_load(graphs, rate=500.0, n_requests=requests, n_warmup=warmup, seed=500,
                          max_slots=4, pool_bytes=48 << 30,
                          progress=lambda d, t: log(f"serving: {d}/{t} requests done"))
    stats["graphs"] = names
    stats["latency"] = "arrival to result visible on the host"
    # the same mix offered below the measured capacity, for latency without
    # queue growth
    low_rate = max(10.0, 0.6 * stats["throughput_rps"])
    low, _ = run_load(graphs, rate=low_rate, n_requests=max(200, requests // 5),
                      n_warmup=max(20, warmup // 5), seed=501, max_slots=4, pool_bytes=48 << 30,
                      progress=lambda d, t: log(f"serving (below capacity): {d}/{t} requests done"))
    stats["below_capacity"] = {k: low[k] for k in ("offered_rate", "requests", "throughput_rps",
                                                   "p50_ms", "p99_ms", "mean_queue_ms", "failed",
                                                   "per_query")}
    log("serving: served vs plain")
    stats["served_vs_plain"] = serve_compare(gpm, torch, graphs)
    return stats


def c4_wedges(off, adj):
    """Wedges x - y - z the 4-cycle kernels scan: y below x and z below x in
    the degree order (x the cycle's top vertex), z != x.  For each arc
    y -> x (y below x) that is the number of y's neighbours ranked below x,
    i.e. x's position among y's neighbours sorted by rank."""
    n = off.shape[0] - 1
    deg = np.diff(off).astype(np.int64)
    rank_key = deg * (1 << 32) + np.arange(n, dtype=np.int64)      # (degree, id)
    rows = np.repeat(np.arange(n, dtype=np.int64), deg)
    key = rank_key[adj.astype(np.int64)]
    # positions within each row after sorting the row by rank
    order = np.lexsort((key, rows))
    pos = np.empty_like(order)
    pos[order] = np.arange(order.shape[0]) - np.repeat(off[:-1].astype(np.int64), deg)
    up = key > rank_key[rows]                    # arcs y -> x with x above y
    return int(pos[up].sum()), int(up.sum())


def motif_leg(gpm, torch, scale=18, cap=1 << 26, reps=3):
    """The motif and listing workload: RMAT-`scale` (seed = scale), induced
    3- and 4-motif counts (local counting) and edge-induced diamond and
    4-cycle listing into a `cap`-row buffer (total and checksum over every
    embedding).  Each call timed with HIP events on its stream; the 4-motif
    call's kernels from the library's timing spans; the 4-cycle kernels
    against the HBM roofline on the bytes of the wedges they scan."""
    import graphgen
    e = graphgen.rmat(scale, seed=scale)
    g = gpm.Graph.build(e.n, torch.from_numpy(e.u).cuda(), torch.from_numpy(e.v).cuda())
    stream = torch.cuda.current_stream()
    gold = {}
    gp = os.path.join(ROOT, "tests", "golden", "rmat_counts.json")
    if os.path.exists(gp):
        with open(gp) as f:
            gold = json.load(f).get(f"rmat{scale}", {})

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            out = fn()
        b.record(stream)
        torch.cuda.synchronize()
        return out, a.elapsed_time(b) / reps

    res = {"workload": f"rmat{scale}: induced 3-/4-motif counts, edge-induced diamond and "
                       f"4-cycle listing (buffer {cap} rows)", "m": g.m}
    ws3 = torch.empty(gpm.binding.motif_workspace_bytes(g, 3), dtype=torch.uint8, device="cuda")
    ws4 = torch.empty(gpm.binding.motif_workspace_bytes(g, 4), dtype=torch.uint8, device="cuda")
    o3 = torch.zeros(3, dtype=torch.int64, device="cuda")
    o4 = torch.zeros(7, dtype=torch.int64, device="cuda")
    _, ms3 = timed(lambda: gpm.motif_count(g, 3, ws=ws3, out=o3))
    _, ms4 = timed(lambda: gpm.motif_count(g, 4, ws=ws4, out=o4))
    m3 = [int(x) for x in o3.tolist()]
    m4 = [int(x) for x in o4.tolist()]
    res["motif3"] = {"counts": m3[:2], "status_word": m3[2], "ms": ms3,
                     "edges_per_sec": g.m / (ms3 * 1e-3),
                     "equals_golden": m3[:2] == gold.get("motif3")}
    res["motif4"] = {"counts": m4[:6], "status_word": m4[6], "ms": ms4,
                     "edges_per_sec": g.m / (ms4 * 1e-3),
                     "equals_golden": m4[:6] == gold.get("motif4")}
    # the 4-motif call's kernels
    torch.cuda.synchronize()
    gpm.timing_enable(True)
    gpm.motif_count(g, 4, ws=ws4, out=o4)
    torch.cuda.synchronize()
    gpm.timing_enable(False)
    phases = {}
    for name, ms, _ in gpm.timing_read():
        phases[name] = phases.get(name, 0.0) + ms
    res["motif4"]["phases_ms"] = {k: round(x, 4) for k, x in phases.items()}
    off_h = g.csr()[0].cpu().numpy().astype(np.int64)
    adj_h = g.csr()[1].cpu().numpy()
    wedges, arcs_up = c4_wedges(off_h, adj_h)
    c4_ms = sum(x for k, x in phases.items() if k.startswith("k_c4"))
    b_c4 = 4 * wedges + 12 * arcs_up
    res["motif4"]["c4_roofline"] = {
        "kernels": sorted(k for k in phases if k.startswith("k_c4")), "bound": "hbm",
        "alg_bytes": b_c4, "wedges": wedges, "ms": c4_ms,
        "achieved": b_c4 / (c4_ms * 1e-3) / 1e9 if c4_ms > 0 else None, "unit": "GB/s",
        "peak": HBM_PEAK_GBS,
        "frac": b_c4 / (c4_ms * 1e-3) / 1e9 / HBM_PEAK_GBS if c4_ms > 0 else None,
        "bytes_model": "4 B per scanned wedge x - y - z (the rank of z, in the graph "
                       "relabelled by degree order) + 12 B per arc y -> x (the middle and its "
                       "segment of the part table); wedges counted under the (degree, id) "
                       "order, the kernels break degree ties in any order"}
    for name, lpat in (("diamond", gpm.diamond(gpm.EDGE_INDUCED | gpm.LIST)),
                       ("4-cycle", gpm.cycle4(gpm.EDGE_INDUCED | gpm.LIST))):
        wsl = torch.empty(gpm.workspace_bytes(g, lpat), dtype=torch.uint8, device="cuda")
        (t, w, c, _), ms = timed(lambda: gpm.list_embeddings(g, lpat, cap, ws=wsl))
        want = gold.get(f"sl_{name}", {})
        res[f"list_{name}"] = {"total": t, "written": w, "checksum": c, "ms": ms,
                               "embeddings_per_sec": t / (ms * 1e-3),
                               "equals_golden": (t, c) == (want.get("total"),
                                                           want.get("checksum"))}
        torch.cuda.empty_cache()
    return res


def generic_leg(gpm, torch, scale, reps=3):
    """The general-pattern plan on two patterns whose counts the local-count
    route also gives, the vertex-induced 4-cycle and 4-path on RMAT-`scale`,
    with and without the per-wave connectivity map."""
    import graphgen
    e = graphgen.rmat(scale, seed=scale)
    g = gpm.Graph.build(e.n, torch.from_numpy(e.u).cuda(), torch.from_numpy(e.v).cuda())

    def timed(fn):
        out = fn()   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            out = fn()
        torch.cuda.synchronize()
        return out, (time.perf_counter() - t0) * 1e3 / reps

    mc, lc_ms = timed(lambda: gpm.motif_count(g, 4))
    names = list(gpm.MOTIF4_NAMES)
    res = {"workload": f"rmat{scale}: vertex-induced 4-cycle and 4-path, general plan "
                       f"(k_generic) vs the 4-motif local-count route",
           "m": g.m, "lc_route_ms_all_six_motifs": lc_ms}
    for name, edges in (("4-cycle", [(0, 1), (1, 2), (2, 3), (3, 0)]),
                        ("4-path", [(0, 1), (1, 2), (2, 3)])):
        p = gpm.pattern(4, edges, gpm.VERTEX_INDUCED)
        got, ms = timed(lambda: gpm.count(g, p))
        # the same plan taking adjacency from binary searches in the matched
        # vertices' rows instead of the connectivity map
        os.environ["GPM_MNC"] = "0"
        try:
            got_off, ms_off = timed(lambda: gpm.count(g, p))
        finally:
            del os.environ["GPM_MNC"]
        # and without degree filtering
        os.environ["GPM_DF"] = "0"
        try:
            got_nodf, ms_nodf = timed(lambda: gpm.count(g, p))
        finally:
            del os.environ["GPM_DF"]
        res[name] = {"count": got, "equals_motif_count": got == mc[names.index(name)],
                     "ms": ms, "matches_per_sec": got / (ms * 1e-3),
                     "ms_without_connectivity_map": ms_off, "same_without_map": got == got_off,
                     "ms_without_degree_filter": ms_nodf,
                     "same_without_degree_filter": got == got_nodf,
                     "lc_route_speedup": ms / lc_ms}
    # listing the 4-cycles: every embedding hashed into the checksum, the
    # first 2^20 written out
    pl = gpm.pattern(4, [(0, 1), (1, 2), (2, 3), (3, 0)], gpm.VERTEX_INDUCED | gpm.LIST)
    ws = torch.empty(gpm.workspace_bytes(g, pl), dtype=torch.uint8, device="cuda")
    (t, w, c, _), lms = timed(lambda: gpm.list_embeddings(g, pl, 1 << 20, ws=ws))
    res["4-cycle listing"] = {"total": t, "written": w, "ms": lms,
                              "equals_count": t == res["4-cycle"]["count"],
                              "embeddings_per_sec": t / (lms * 1e-3)}
    return res


def large_k_leg(gpm, torch, plan=((12, 9), (16, 8), (18, 7), (20, 6))):
    """k-clique counts for growing k (the paper's large-pattern experiment):
    for each (scale, kmax), RMAT-`scale` and k = 4..kmax, one timed
    gpm_count call each (after a warm-up call for k <= 6; the larger k run
    for seconds, where a launch's start-up cost does not show)."""
    import graphgen
    out = []
    for scale, kmax in plan:
        e = graphgen.rmat(scale, seed=scale)
        g = gpm.Graph.build(e.n, torch.from_numpy(e.u).cuda(), torch.from_numpy(e.v).cuda())
        for k in range(4, kmax + 1):
            p = gpm.clique(k)
            if k <= 6:
                gpm.count(g, p)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            c = gpm.count(g, p)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            log(f"rmat{scale} {k}-cliques: {c} in {ms:.1f} ms")
            out.append({"scale": scale, "k": k, "count": c, "ms": ms,
                        "cliques_per_sec": c / (ms * 1e-3)})
    return {"workload": "k-clique counts on RMAT graphs for growing k", "runs": out}


def core_orient_leg(gpm, torch, scale=20, reps=3):
    """The core-value orientation on RMAT-`scale`: the device core
    decomposition and DAG rebuild (gpm_graph_orient), then the 3-/4-/5-clique
    counts under each orientation."""
    import graphgen
    e = graphgen.rmat(scale, seed=scale)
    g = gpm.Graph.build(e.n, torch.from_numpy(e.u).cuda(), torch.from_numpy(e.v).cuda())

    def cliques():
        out = {}
        for k in (3, 4, 5):
            p = gpm.clique(k)
            gpm.count(g, p)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                c = gpm.count(g, p)
            torch.cuda.synchronize()
            out[f"clique{k}"] = {"count": c, "ms": (time.perf_counter() - t0) * 1e3 / reps}
        return out

    def orient_ms(order):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = g.orient(order, core_out=order == gpm.ORIENT_CORE)
        torch.cuda.synchronize()
        return out, (time.perf_counter() - t0) * 1e3

    res = {"workload": f"rmat{scale}: core-value orientation vs degree orientation"}
    res["degree_order"] = dict(cliques(), max_out_degree=g.max_out_degree)
    orient_ms(gpm.ORIENT_CORE)   # warm-up (first-call set-up)
    orient_ms(gpm.ORIENT_DEGREE)
    core_ms, deg_ms = [], []
    for _ in range(reps):
        core, ms = orient_ms(gpm.ORIENT_CORE)
        core_ms.append(ms)
        deg_ms.append(orient_ms(gpm.ORIENT_DEGREE)[1])
    res["orient_core_ms"] = sum(core_ms) / reps
    res["orient_degree_ms"] = sum(deg_ms) / reps
    res["degeneracy"] = int(core.max()) if g.n else 0
    g.orient(gpm.ORIENT_CORE)
    res["core_order"] = dict(cliques(), max_out_degree=g.max_out_degree)
    g.orient(gpm.ORIENT_DEGREE)
    res["same_counts"] = all(res["degree_order"][f"clique{k}"]["count"] ==
                             res["core_order"][f"clique{k}"]["count"] for k in (3, 4, 5))
    return res


def local_graph_leg(gpm, torch, scale, reps=3):
    """4- and 5-clique counts on RMAT-`scale` through the local-graph
    kernels (the default) and through the depth-first search without local
    graphs (GPM_LG=0): the search on a local graph of the paper, as an
    ablation."""
    import graphgen
    e = graphgen.rmat(scale, seed=scale)
    g = gpm.Graph.build(e.n, torch.from_numpy(e.u).cuda(), torch.from_numpy(e.v).cuda())

    def timed(fn):
        out = fn()   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            out = fn()
        torch.cuda.synchronize()
        return out, (time.perf_counter() - t0) * 1e3 / reps

    res = {"workload": f"rmat{scale}: 4- and 5-clique counts with and without local graphs",
           "m": g.m}
    for k in (4, 5):
        p = gpm.clique(k)
        c, ms = timed(lambda: gpm.count(g, p))
        os.environ["GPM_LG"] = "0"
        try:
            c_off, ms_off = timed(lambda: gpm.count(g, p))
        finally:
            del os.environ["GPM_LG"]
        res[f"clique{k}"] = {"count": c, "ms": ms, "ms_without_local_graphs": ms_off,
                             "same": c == c_off, "local_graph_speedup": ms_off / ms}
    return res


def formula_scale_leg(gpm, torch, scales=(10, 11, 12, 13, 14, 15, 16), reps=3):
    """The 5-motif formula route alone on RMAT-10 .. RMAT-16 (RMAT-16: 65,536
    vertices, the largest graph whose rows of A^2 fit in LDS): call time (one
    warm-up, `reps` timed calls) and the per-kernel spans."""
    import graphgen

    out = []
    for sc in scales:
        e = graphgen.rmat(sc, seed=sc)
        g = gpm.Graph.build(e.n, torch.from_numpy(e.u).cuda(), torch.from_numpy(e.v).cuda())
        ws = torch.empty(gpm.motif_formula_workspace_bytes(g, 5), dtype=torch.uint8,
                         device="cuda")
        c = gpm.motif_count_formula(g, 5, ws=ws)
        torch.cuda.synchronize()
        gpm.timing_enable(True)
        t0 = time.perf_counter()
        for _ in range(reps):
            c = gpm.motif_count_formula(g, 5, ws=ws)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        gpm.timing_enable(False)
        spans = {}
        for name, t, _ in gpm.timing_read():
            if name.startswith("k_f5"):
                spans[name] = round(spans.get(name, 0.0) + t / reps, 3)
        out.append({"graph": f"rmat{sc}", "n": g.n, "m": g.m, "ms": ms,
                    "connected_5_subgraphs": sum(c),
                    "subgraphs_per_sec": sum(c) / (ms * 1e-3), "spans_ms": spans})
    return out


def motif_enum_leg(gpm, torch, scale4=12, scale5=10, reps=3, enum5_large=False):
    """Pattern-oblivious motif counting (vertex extension of canonical
    embeddings, connectivity codes; no counting formulas): the 4-motifs of
    RMAT-`scale4` against the local-count route's time for the same six
    counts, and the 21 5-motifs of RMAT-`scale5` against the formula route
    (which also runs on RMAT-`scale4`; with `enum5_large`, one enumeration
    call there too, about 5 s)."""
    import graphgen

    def timed(fn):
        out = fn()   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            out = fn()
        torch.cuda.synchronize()
        return out, (time.perf_counter() - t0) * 1e3 / reps

    def without_map(fn):
        # the same kernel taking connectivity from binary searches in the
        # embedding's rows instead of the per-wave connectivity map
        os.environ["GPM_MNC"] = "0"
        try:
            return timed(fn)
        finally:
            del os.environ["GPM_MNC"]

    e = graphgen.rmat(scale4, seed=scale4)
    g = gpm.Graph.build(e.n, torch.from_numpy(e.u).cuda(), torch.from_numpy(e.v).cuda())
    ws = torch.empty(gpm.motif_enum_workspace_bytes(g, 4), dtype=torch.uint8, device="cuda")
    run4 = lambda: gpm.motif_count_enum(g, 4, ws=ws)   # noqa: E731
    c4, ms4 = timed(run4)
    c4_off, ms4_off = without_map(run4)
    lc4, lc_ms = timed(lambda: gpm.motif_count(g, 4))
    e5 = graphgen.rmat(scale5, seed=scale5)
    g5 = gpm.Graph.build(e5.n, torch.from_numpy(e5.u).cuda(), torch.from_numpy(e5.v).cuda())
    ws5 = torch.empty(gpm.motif_enum_workspace_bytes(g5, 5), dtype=torch.uint8, device="cuda")
    run5 = lambda: gpm.motif_count_enum(g5, 5, ws=ws5)   # noqa: E731
    c5, ms5 = timed(run5)
    c5_off, ms5_off = without_map(run5)
    # the formula route for the same 21 counts (closed forms in local counts
    # for fifteen classes, the rows of A^2 and the triangles for four more,
    # the 4-cycles in each neighbourhood for the wheel, the clique kernels
    # for K5, back-substitution)
    wsf = torch.empty(gpm.motif_formula_workspace_bytes(g5, 5), dtype=torch.uint8, device="cuda")
    f5, msf = timed(lambda: gpm.motif_count_formula(g5, 5, ws=wsf))
    wsf12 = torch.empty(gpm.motif_formula_workspace_bytes(g, 5), dtype=torch.uint8,
                        device="cuda")
    f12, msf12 = timed(lambda: gpm.motif_count_formula(g, 5, ws=wsf12))
    large = {"ms": msf12, "subgraphs_per_sec": sum(f12) / (msf12 * 1e-3), "counts": f12}
    if enum5_large:
        del wsf12
        ws12 = torch.empty(gpm.motif_enum_workspace_bytes(g, 5), dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c12 = gpm.motif_count_enum(g, 5, ws=ws12)
        torch.cuda.synchronize()
        large["enumeration_ms_one_call"] = (time.perf_counter() - t0) * 1e3
        large["enumeration_equals_formula"] = c12 == f12
        large["formula_speedup"] = large["enumeration_ms_one_call"] / msf12
    return {"workload": f"rmat{scale4} 4-motifs and rmat{scale5} 5-motifs by enumeration "
                        f"(k_motif_enum) vs the 4-motif local-count route and the 5-motif "
                        f"formula route",
            "motif4": {"counts": c4, "equals_local_count_route": c4 == lc4, "ms": ms4,
                       "subgraphs_per_sec": sum(c4) / (ms4 * 1e-3),
                       "ms_without_connectivity_map": ms4_off, "same_without_map": c4 == c4_off,
                       "local_count_route_ms": lc_ms, "local_count_speedup": ms4 / lc_ms},
            "motif5": {"counts": c5, "ms": ms5, "subgraphs_per_sec": sum(c5) / (ms5 * 1e-3),
                       "ms_without_connectivity_map": ms5_off,
                       "same_without_map": c5 == c5_off,
                       "formula_route_ms": msf, "formula_equals_enumeration": f5 == c5,
                       "formula_speedup": ms5 / msf},
            f"motif5_formula_rmat{scale4}": large}


def tune_leg(gpm, torch, g, pats, ks, skip, reps=5):
    """Per-graph tuning of the plain path's task granularity (untimed set-up,
    once per graph): gpm_graph_autotune on the workload's graph, then each
    clique count timed under the default and the chosen setting."""
    default = g.tuning()
    res = {"default": default}
    if skip:
        res["chosen"] = default
        return res
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    chosen = g.autotune()
    torch.cuda.synchronize()
    res["autotune_ms"] = (time.perf_counter() - t0) * 1e3
    res["chosen"] = chosen

    def per_count(t):
        g.set_tuning(**t)
        out = {}
        for k, p in zip(ks, pats):
            c = gpm.count(g, p)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(reps):
                c = gpm.count(g, p)
            torch.cuda.synchronize()
            out[f"clique{k}"] = {"count": c, "ms": (time.perf_counter() - t1) * 1e3 / reps}
        return out

    res["ms_default"] = per_count(default)
    res["ms_chosen"] = per_count(chosen)
    res["same_counts"] = all(res["ms_default"][x]["count"] == res["ms_chosen"][x]["count"]
                             for x in res["ms_default"])
    g.set_tuning(**chosen)
    return res


# The paper's own CPU figures (Sec. 6: input-graph table, TC and k-clique
# tables), context only: real graphs, another machine, no RMAT.  #E counts
# arcs, so undirected edges/s = (#E / 2) / time.
PAPER_CONTEXT = {
    "machine": "4-socket Intel Xeon Gold 5120, 2.2 GHz, 56 cores, 56 threads, 190 GB",
    "graphs_arcs": {"Lj": 86e6, "Or": 234e6, "Tw4": 2405e6, "Fr": 3612e6, "Uk": 6604e6},
    "tc_seconds_hi": {"Lj": 0.3, "Or": 1.8, "Tw4": 57.2, "Fr": 44.9, "Uk": 24.5},
    "clique4_seconds_hi_lo": {"Lj": [0.6, 0.7], "Or": [2.4, 1.9], "Tw4": [1676.8, 681.8],
                              "Fr": [166.2, 60.4], "Uk": [2481.2, 2451.7]},
    "clique5_seconds_hi_lo": {"Lj": [13.9, 14.2], "Or": [7.4, 4.8], "Fr": [194.9, 64.3]},
}


def paper_context():
    c = dict(PAPER_CONTEXT)
    arcs = c["graphs_arcs"]
    c["tc_edges_per_sec_hi"] = {k: arcs[k] / 2 / t for k, t in c["tc_seconds_hi"].items()}
    c["clique4_edges_per_sec_lo"] = {k: arcs[k] / 2 / t[1]
                                     for k, t in c["clique4_seconds_hi_lo"].items()}
    c["note"] = "the paper's numbers on its machine and graphs; not this workload, not a target"
    return c


def copy_calibration():
    import torch
    n = 1 << 30
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "copies": 3}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scale", type=int, default=20)
    ap.add_argument("--kmax", type=int, default=5, help="largest clique size counted")
    ap.add_argument("--cpu-fraction", type=int, default=48,
                    help="the CPU baseline times every F-th root")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default task granularity instead of tuning it on the graph")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-graphs", type=int, default=20000)
    ap.add_argument("--plain-graphs", type=int, default=2000,
                    help="graphs timed for the general per-graph call (scaled to all)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=5000)
    ap.add_argument("--serve-warmup", type=int, default=500)
    ap.add_argument("--no-generic", action="store_true")
    ap.add_argument("--no-motif-enum", action="store_true")
    ap.add_argument("--no-lg-ablation", action="store_true")
    ap.add_argument("--core-only", action="store_true",
                    help="only time the core-value orientation on RMAT-20 and exit")
    ap.add_argument("--large-k-only", action="store_true",
                    help="only count k-cliques for k = 4..9 on RMAT-12/16/18/20 (minutes) and exit")
    ap.add_argument("--lg-ablation-only", action="store_true",
                    help="time only the local-graph ablation leg (for kernel traces) and exit")
    ap.add_argument("--motif-enum-only", action="store_true",
                    help="time only the pattern-oblivious motif leg (for kernel traces) and exit")
    ap.add_argument("--enum5-large", action="store_true",
                    help="with --motif-enum-only: also time one 5-motif enumeration of "
                         "RMAT-12 (about 5 s) against the formula route")
    ap.add_argument("--formula-only", action="store_true",
                    help="time only the 5-motif formula route on RMAT-10 .. RMAT-16 and exit")
    ap.add_argument("--motif-only", action="store_true",
                    help="time only the RMAT-18 motif and listing leg (for kernel traces) and exit")
    ap.add_argument("--no-motif", action="store_true")
    ap.add_argument("--generic-only", action="store_true",
                    help="time only the general-pattern leg (for kernel traces) and exit")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB device to device three times (reference kernel "
                         "for scaling hardware byte counters) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the design for more GPUs is written up, not built).", file=sys.stderr)
        sys.exit(2)

    import torch
    import graphgen
    import paper_2011_03135_amd as gpm

    gpm.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.generic_only:
        print(json.dumps({"generic_pattern": generic_leg(gpm, torch, 13)}))
        return
    if args.motif_only:
        print(json.dumps({"motifs_listing": motif_leg(gpm, torch)}))
        return
    if args.core_only:
        print(json.dumps({"core_orientation": core_orient_leg(gpm, torch)}))
        return
    if args.large_k_only:
        print(json.dumps({"large_k_cliques": large_k_leg(gpm, torch)}))
        return
    if args.lg_ablation_only:
        print(json.dumps({"local_graph_ablation": local_graph_leg(gpm, torch, 14)}))
        return
    if args.formula_only:
        print(json.dumps({"formula_scaling": formula_scale_leg(gpm, torch)}))
        return
    if args.motif_enum_only:
        print(json.dumps({"motif_enumeration": motif_enum_leg(gpm, torch,
                                                              enum5_large=args.enum5_large)}))
        return
    e = graphgen.rmat(args.scale, seed=args.scale)
    u = torch.from_numpy(e.u).to(dev)
    v = torch.from_numpy(e.v).to(dev)
    gb, sb = gpm.Graph.build_bytes(e.n, e.u.shape[0])
    storage = torch.empty(gb, dtype=torch.uint8, device=dev)
    scratch = torch.empty(sb, dtype=torch.uint8, device=dev)
    ks = list(range(3, args.kmax + 1))
    pats = [gpm.clique(k) for k in ks]
    g0 = gpm.Graph.build(e.n, u, v, storage=storage, scratch=scratch)
    m = g0.m
    off_h = g0.csr()[0].cpu().numpy().astype(np.int64)
    adj_h = g0.csr()[1].cpu().numpy()
    out = torch.zeros(len(ks), dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()
    tuning = tune_leg(gpm, torch, g0, pats, ks, args.no_autotune)
    # the tuning can shrink the triangle chunks: size the workspace after it
    wsb = max([gpm.workspace_bytes(g0, p) for p in pats]
              + [gpm.binding.clique_counts_workspace_bytes(g0, args.kmax)])
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)

    def step():
        # the step: device CSR build + orientation, then every clique count of
        # the workload in one local-graph pass (under the graph's tuning)
        g = gpm.Graph.build(e.n, u, v, storage=storage, scratch=scratch)
        g.set_tuning(**tuning["chosen"])
        if args.kmax >= 4:
            gpm.clique_counts(g, args.kmax, ws=ws, out=out)
        else:
            gpm.count(g, pats[0], ws=ws, out=out)
        return g

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    gpm.timing_enable(True)
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    t_start.record(stream)
    for i in range(args.steps):
        g = step()
    t_end.record(stream)
    torch.cuda.synchronize()
    gpm.timing_enable(False)
    spans = gpm.timing_read()
    ms_step = t_start.elapsed_time(t_end) / args.steps
    counts = [int(x) for x in out.tolist()]
    log(f"timed {args.steps} steps: {ms_step:.2f} ms/step")

    # each counting call on its own (one call per size, as a user counting a
    # single pattern would), HIP events around each call
    names = ["graph_build"] + [f"clique{k}" for k in ks]
    phase_ms = [0.0] * len(names)
    sep = torch.zeros(len(ks), dtype=torch.int64, device=dev)
    for it in range(args.warmup + args.steps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)]
        ev[0].record(stream)
        g = gpm.Graph.build(e.n, u, v, storage=storage, scratch=scratch)
        g.set_tuning(**tuning["chosen"])
        ev[1].record(stream)
        for i, p in enumerate(pats):
            gpm.count(g, p, ws=ws, out=sep[i:i + 1])
            ev[i + 2].record(stream)
        torch.cuda.synchronize()
        if it >= args.warmup:
            for i in range(len(names)):
                phase_ms[i] += ev[i].elapsed_time(ev[i + 1]) / args.steps
    sep_counts = [int(x) for x in sep.tolist()]

    phases, units = {}, {}
    for name, ms, un in spans:
        phases[name] = phases.get(name, 0.0) + ms / args.steps
        units[name] = units.get(name, 0) + un / args.steps
    dom = max((k for k in phases if k != "graph_build"), key=lambda k: phases[k])
    roof = roofline(dom, phases[dom], int(units[dom]), off_h, adj_h,
                    tuning["chosen"]["lg5_slice"])
    per_problem = {"graph_build": {"ms": phase_ms[0]}}
    for k, c, ms in zip(ks, sep_counts, phase_ms[1:]):
        per_problem[f"{k}-clique" if k > 3 else "TC"] = {
            "ms": ms, "edges_per_sec": m / (ms * 1e-3), "matches_per_sec": c / (ms * 1e-3)}
    per_problem["separate_calls_equal_fused"] = sep_counts == counts
    phase_roof = {}
    if 3 in ks:
        phase_roof["TC"] = phase_roofline("TC", phase_ms[1 + ks.index(3)], off_h, adj_h, 2)
    if 4 in ks:
        phase_roof["4-clique"] = phase_roofline("4-clique", phase_ms[1 + ks.index(4)], off_h,
                                                adj_h, 3)

    res = {
        "metric": "edges/sec & matches/sec for TC and 4-clique on RMAT-20; batched vs plain speedup",
        "value": m / (ms_step * 1e-3),
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {
            "workload": f"rmat{args.scale}: device CSR build + degree-ordered DAG + "
                        + ", ".join(f"{k}-clique" for k in ks) + " counts in one local-graph pass",
            "n": e.n, "m": m, "input_edges": int(e.u.shape[0]), "seed": args.scale,
            "rmat_abcd": [0.57, 0.19, 0.19, 0.05],
        },
        "counts": {f"clique{k}": c for k, c in zip(ks, counts)},
        "matches_per_sec": sum(counts) / (ms_step * 1e-3),
        "count_phase_edges_per_sec": m / ((ms_step - phases.get("graph_build", 0.0)) * 1e-3),
        "per_problem": per_problem,
        "phases_ms": {k: round(x, 4) for k, x in phases.items()},
        "roofline": roof,
        "phase_rooflines": phase_roof,
        "tuning": tuning,
        "paper_context": paper_context(),
    }
    if not args.no_batch:
        res["batched_vs_plain"] = batch_leg(gpm, torch, args.batch_graphs, args.plain_graphs, 20)
    if not args.no_motif:
        log("motifs and listing (rmat18)")
        res["motifs_listing"] = motif_leg(gpm, torch)
    if not args.no_generic:
        log("general pattern")
        res["generic_pattern"] = generic_leg(gpm, torch, 13)
    if not args.no_motif_enum:
        log("motif enumeration")
        res["motif_enumeration"] = motif_enum_leg(gpm, torch)
    if not args.no_lg_ablation:
        log("local-graph ablation")
        res["local_graph_ablation"] = local_graph_leg(gpm, torch, 14)
    if not args.no_serve:
        log("serving load")
        g_res = gpm.Graph.build(e.n, u, v)
        res["serving"] = serve_leg(gpm, torch, g_res, args.scale, args.serve_requests,
                                   args.serve_warmup)
    if not args.no_cpu_baseline:
        log("cpu baseline")
        threads = len(os.sched_getaffinity(0))
        res["cpu_baseline"] = cpu_baseline(e, args.cpu_fraction, ks, threads, counts)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
