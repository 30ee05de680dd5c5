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


def test_batch_graph_capture_replays(gpm):
    batch = graphgen.rgg_batch(500, seed=99)
    g, voff = union_graph(gpm, batch)
    eager = gpm.batch_motif_count(g, voff, 4).clone()
    out = torch.zeros_like(eager)
    ws = torch.empty(1 << 16, dtype=torch.uint8, device="cuda")
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
