"""Batched per-graph motif counts (one fused launch) against the oracle."""
import numpy as np
import pytest
import torch

import graphgen
import oracle
from gpu_util import build

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpm():
    import paper_2011_03135_amd as m
    m.load()
    return m


def union_graph(gpm, batch):
    e = graphgen.EdgeList(batch.n, batch.u, batch.v)
    g = build(gpm, e)
    voff = torch.from_numpy(batch.voff.astype(np.int32)).cuda()
    return g, voff


def unpack(t):
    return [[int(x) + (1 << 64) if int(x) < 0 else int(x) for x in row] for row in t.cpu().tolist()]


@pytest.mark.parametrize("k", [3, 4])
def test_batch_rgg_vs_oracle(gpm, k):
    batch = graphgen.rgg_batch(300, seed=2020)
    g, voff = union_graph(gpm, batch)
    got = unpack(gpm.batch_motif_count(g, voff, k))
    want = oracle.batch_motifs(batch, k)
    for i in range(batch.num_graphs):
        assert got[i][-1] == 0, (i, got[i])
        assert got[i][:-1] == want[i], i


def test_batch_mixed_sizes_and_errors(gpm):
    parts = [graphgen.erdos_renyi(300, 0.05, 1),          # > 256 vertices: workgroup kernel
             graphgen.complete_graph(6),
             graphgen.EdgeList(1, np.zeros(0, np.int32), np.zeros(0, np.int32)),
             graphgen.complete_bipartite(20, 30),
             graphgen.erdos_renyi(1100, 0.003, 2)]        # too large for the batch path
    u = graphgen.disjoint_union(parts)
    voff = np.cumsum([0] + [p.n for p in parts]).astype(np.int32)
    g = build(gpm, u)
    got = unpack(gpm.batch_motif_count(g, torch.from_numpy(voff).cuda(), 4))
    for i, p in enumerate(parts[:4]):
        off, adj = oracle.canonical_csr(p.n, p.u, p.v)
        assert got[i][-1] == 0
        assert got[i][:6] == oracle.motif4(off, adj)
    assert got[4][-1] == 64
    # an edge that joins graphs 1 and 2 is reported, not miscounted silently
    bad = graphgen.disjoint_union(parts[:4])
    bad = graphgen.EdgeList(bad.n, np.append(bad.u, np.int32(300)), np.append(bad.v, np.int32(306)))
    gb = build(gpm, bad)
    got = unpack(gpm.batch_motif_count(gb, torch.from_numpy(voff[:5]).cuda(), 4))
    assert got[1][-1] & 256 and got[2][-1] & 256


def test_batch_equals_plain(gpm):
    batch = graphgen.rgg_batch(12, seed=7)
    g, voff = union_graph(gpm, batch)
    got = unpack(gpm.batch_motif_count(g, voff, 4))
    for i in range(batch.num_graphs):
        gi = build(gpm, batch.graph(i))
        assert got[i][:6] == gpm.motif_count(gi, 4)


def test_batch_sub_ranges(gpm):
    """d_voff may point into the union's offset array: one graph (G = 1) or
    a run of graphs mined alone give the full batch's rows for them."""
    batch = graphgen.rgg_batch(60, seed=21)
    g, voff = union_graph(gpm, batch)
    full = gpm.batch_motif_count(g, voff, 4)
    for i in (0, 7, 59):
        one = gpm.batch_motif_count(g, voff[i:i + 2], 4)
        assert torch.equal(one[0], full[i]), i
    run = gpm.batch_motif_count(g, voff[10:31], 4)
    assert torch.equal(run, full[10:30])


def test_batch_graph_capture_replays(gpm):
    batch = graphgen.rgg_batch(500, seed=99)
    g, voff = union_graph(gpm, batch)
    eager = gpm.batch_motif_count(g, voff, 4).clone()
    out = torch.zeros_like(eager)
    wsb = gpm.binding.batch_workspace_bytes(batch.num_graphs, 4)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        gpm.batch_motif_count(g, voff, 4, ws=ws, out=out)   # warm up outside capture
    torch.cuda.current_stream().wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        gpm.batch_motif_count(g, voff, 4, ws=ws, out=out)
    for r in range(4):
        out.zero_()
        junk = torch.randn(1000, device="cuda").sum()   # eager work between replays
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), r
        del junk


def test_batch_full_workload(gpm):
    """20,000 random geometric graphs (n uniform in [10, 200]), seed 2020."""
    batch = graphgen.rgg_batch(20000, seed=2020)
    g, voff = union_graph(gpm, batch)
    got = unpack(gpm.batch_motif_count(g, voff, 4))
    want = oracle.batch_motifs(batch, 4)
    assert all(r[-1] == 0 for r in got)
    assert [r[:6] for r in got] == want


def tier_parts():
    """Graphs on both sides of every tier bound (64, 128, 256, 1024 vertices)."""
    sizes = [1, 2, 63, 64, 65, 127, 128, 129, 255, 256, 257, 700, 1024]
    parts = []
    for i, n in enumerate(sizes):
        p = min(1.0, 8.0 / max(n - 1, 1))
        parts.append(graphgen.erdos_renyi(n, p, 100 + i))
    parts.insert(5, graphgen.complete_graph(40))
    parts.insert(9, graphgen.complete_bipartite(60, 60))
    return parts


def all_configs(gpm):
    out = []
    for nt in (64, 128, 256):
        for tiers in (1, 2, 3):
            for bpc in (4, 8, 16, 32):
                out.append(gpm.BatchConfig(nt, tiers, bpc, 0))
    return out


@pytest.fixture(scope="module")
def tier_batch(gpm):
    parts = tier_parts()
    u = graphgen.disjoint_union(parts)
    voff = np.cumsum([0] + [p.n for p in parts]).astype(np.int32)
    want = []
    for p in parts:
        off, adj = oracle.canonical_csr(p.n, p.u, p.v)
        want.append(oracle.motif4(off, adj, 8))
    return build(gpm, u), torch.from_numpy(voff).cuda(), want


def test_batch_every_config_matches_oracle(gpm, tier_batch):
    g, voff, want = tier_batch
    for cfg in all_configs(gpm):
        got = unpack(gpm.batch_motif_count(g, voff, 4, config=cfg))
        assert [r[-1] for r in got] == [0] * len(want), cfg.as_dict()
        assert [r[:6] for r in got] == want, cfg.as_dict()


def test_batch_autotune(gpm, tier_batch):
    g, voff, want = tier_batch
    best, ms, out = gpm.batch_autotune(g, voff, 4, reps=2)
    assert ms > 0
    assert best.as_dict() in [c.as_dict() for c in all_configs(gpm)]
    assert [r[:6] for r in unpack(out)] == want
    # the default configuration is one of the candidates
    assert gpm.batch_default_config().as_dict() in [c.as_dict() for c in all_configs(gpm)]


def test_batch_bad_config_rejected(gpm, tier_batch):
    g, voff, _ = tier_batch
    for bad in (gpm.BatchConfig(96, 1, 8, 0), gpm.BatchConfig(64, 4, 8, 0),
                gpm.BatchConfig(64, 1, 0, 0), gpm.BatchConfig(64, 1, 33, 0)):
        with pytest.raises(gpm.GpmError):
            gpm.batch_motif_count(g, voff, 4, config=bad)


def test_batch_empty_graphs(gpm):
    """Graphs with no vertices get zero counts and status 0."""
    parts = [graphgen.complete_graph(5), graphgen.cycle_graph(7)]
    u = graphgen.disjoint_union(parts)
    voff = np.array([0, 0, 5, 5, 5, 12, 12], dtype=np.int32)
    g = build(gpm, u)
    got = unpack(gpm.batch_motif_count(g, torch.from_numpy(voff).cuda(), 3))
    assert got == [[0, 0, 0], [0, 10, 0], [0, 0, 0], [0, 0, 0], [7, 0, 0], [0, 0, 0]]

