"""Pattern-oblivious motif counting (k = 3, 4, 5) on the device against the
oracle: the local-counting oracle for k = 3, 4, the oracle's plain
enumeration of each class's pattern for k = 5, brute force on tiny graphs,
and closed forms."""
from itertools import combinations
from math import comb

import numpy as np
import pytest

import brute
import graphgen
import oracle
from gpu_util import build

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpm():
    import paper_2011_03135_amd as m
    m.load()
    return m


def hub_graph():
    """ER(100, 0.06) plus a hub joined to 45 vertices."""
    base = graphgen.erdos_renyi(100, 0.06, 3)
    rng = np.random.default_rng(3)
    ends = rng.choice(np.arange(1, 100), size=45, replace=False).astype(np.int32)
    u = np.concatenate([base.u, np.zeros(45, np.int32)])
    v = np.concatenate([base.v, ends])
    return graphgen.EdgeList(100, u, v, "hub")


def graphs():
    return [graphgen.erdos_renyi(80, 0.1, 1),
            graphgen.erdos_renyi(150, 0.05, 2),
            hub_graph(),
            graphgen.complete_graph(9),
            graphgen.star_graph(40),
            graphgen.relabel(graphgen.complete_bipartite(6, 7), 5)]


@pytest.mark.parametrize("gi", range(6))
def test_3_4_motifs_vs_oracle(gpm, gi):
    e = graphs()[gi]
    print(f"graph {gi} n={e.n}", flush=True)
    g = build(gpm, e)
    off, adj = oracle.canonical_csr(e.n, e.u, e.v)
    assert gpm.motif_count_enum(g, 3) == oracle.motif3(off, adj)
    assert gpm.motif_count_enum(g, 4) == oracle.motif4(off, adj)


@pytest.mark.parametrize("gi", range(6))
def test_5_motifs_vs_oracle(gpm, gi):
    e = graphs()[gi]
    print(f"graph {gi} n={e.n}", flush=True)
    g = build(gpm, e)
    off, adj = oracle.canonical_csr(e.n, e.u, e.v)
    got = gpm.motif_count_enum(g, 5)
    want = [oracle.pattern_count(off, adj, 5, gpm.motif_class_pattern(5, i), True)[0]
            for i in range(21)]
    assert got == want


def test_5_motifs_brute_force(gpm):
    """Every 5-vertex subset of a tiny graph, classified by trying all
    relabellings (no oracle involved)."""
    e = graphgen.erdos_renyi(16, 0.35, 9)
    g = build(gpm, e)
    adj = brute.adjacency_sets(e.n, e.u, e.v)
    forms = [brute.canon(5, gpm.motif_class_pattern(5, i)) for i in range(21)]
    want = [0] * 21
    for vs in combinations(range(e.n), 5):
        ed = brute.induced_edges(adj, vs)
        if brute.connected(5, ed):
            want[forms.index(brute.canon(5, ed))] += 1
    assert gpm.motif_count_enum(g, 5) == want


def test_closed_forms(gpm):
    # K_n: only the clique class, C(n, k) times
    g = build(gpm, graphgen.complete_graph(12))
    for k, top in ((3, 1), (4, 5), (5, 20)):
        want = [0] * gpm.motif_classes(k)
        want[top] = comb(12, k)
        assert gpm.motif_count_enum(g, k) == want
    # star with L leaves: only the (k-1)-star class, C(L, k-1) times
    g = build(gpm, graphgen.star_graph(300))
    for k in (3, 4, 5):
        got = gpm.motif_count_enum(g, k)
        assert got[0] == comb(300, k - 1) and sum(got) == got[0]
    # n-cycle, n >= 6: n paths on k vertices and nothing else
    g = build(gpm, graphgen.cycle_graph(1000))
    paths = {3: 0, 4: 1}   # wedge, 4-path
    for k in (3, 4):
        got = gpm.motif_count_enum(g, k)
        assert got[paths[k]] == 1000 and sum(got) == 1000
    got5 = gpm.motif_count_enum(g, 5)
    p5 = brute.canon(5, [(0, 1), (1, 2), (2, 3), (3, 4)])
    i5 = [brute.canon(5, gpm.motif_class_pattern(5, i)) for i in range(21)].index(p5)
    assert got5[i5] == 1000 and sum(got5) == 1000


def test_edgeless_and_errors(gpm):
    from paper_2011_03135_amd.binding import GpmError
    e = graphgen.EdgeList(5, np.zeros(0, np.int32), np.zeros(0, np.int32), "empty")
    g = build(gpm, e)
    for k in (3, 4, 5):
        assert gpm.motif_count_enum(g, k) == [0] * gpm.motif_classes(k)
    for k in (2, 6):
        with pytest.raises(GpmError) as ei:
            gpm.motif_count_enum(g, k)
        assert ei.value.status == 5


def test_two_routes_agree_rmat(gpm):
    """At sizes beyond the oracle: the enumeration route and the
    local-counting route give the same 3- and 4-motif counts."""
    for scale in (10, 12):
        e = graphgen.rmat(scale, seed=11)
        print(f"rmat {scale}", flush=True)
        g = build(gpm, e)
        assert gpm.motif_count_enum(g, 3) == gpm.motif_count(g, 3)
        assert gpm.motif_count_enum(g, 4) == gpm.motif_count(g, 4)


@pytest.mark.parametrize("gi", [0, 2, 4])
def test_without_connectivity_map(gpm, gi, monkeypatch):
    """GPM_MNC=0 takes the connectivity bits from binary searches in
    the embedding's rows instead of the per-wave map: same counts."""
    e = graphs()[gi]
    print(f"graph {gi} n={e.n}", flush=True)
    g = build(gpm, e)
    off, adj = oracle.canonical_csr(e.n, e.u, e.v)
    monkeypatch.setenv("GPM_MNC", "0")
    assert gpm.motif_count_enum(g, 4) == oracle.motif4(off, adj)
    want = [oracle.pattern_count(off, adj, 5, gpm.motif_class_pattern(5, i), True)[0]
            for i in range(21)]
    assert gpm.motif_count_enum(g, 5) == want


def test_map_on_and_off_agree(gpm, monkeypatch):
    """RMAT-12 (map on by default) and a sparse graph above the map's vertex
    limit (map off): both settings and the local-count route agree."""
    e = graphgen.rmat(12, seed=5)
    g = build(gpm, e)
    on = gpm.motif_count_enum(g, 4)
    monkeypatch.setenv("GPM_MNC", "0")
    assert gpm.motif_count_enum(g, 4) == on == gpm.motif_count(g, 4)
    monkeypatch.delenv("GPM_MNC")
    big = graphgen.erdos_renyi(20000, 6.0 / 20000, 6)
    gb = build(gpm, big)
    assert gpm.motif_count_enum(gb, 4) == gpm.motif_count(gb, 4)
    assert gpm.motif_count_enum(gb, 3) == gpm.motif_count(gb, 3)


def test_union_and_relabel_invariance(gpm):
    """Counts of a disjoint union are the sums of the parts' counts (with
    isolated vertices between them), and relabelling changes nothing."""
    parts = [graphgen.erdos_renyi(60, 0.12, 21), graphgen.complete_graph(7),
             graphgen.EdgeList(9, np.zeros(0, np.int32), np.zeros(0, np.int32), "isolated"),
             hub_graph()]
    for k in (3, 4, 5):
        want = [sum(x) for x in zip(*(gpm.motif_count_enum(build(gpm, p), k)
                                      for p in parts if p.u.shape[0] > 0))]
        union = graphgen.disjoint_union(parts)
        assert gpm.motif_count_enum(build(gpm, union), k) == want
        assert gpm.motif_count_enum(build(gpm, graphgen.relabel(union, 8)), k) == want


def test_graph_capture_replays(gpm):
    """The call records only kernels (fills instead of memsets), so it can be
    captured in a HIP graph and replayed."""
    import torch
    e = graphgen.rmat(11, seed=3)
    g = build(gpm, e)
    for k in (3, 4):
        eager = torch.tensor(gpm.motif_count_enum(g, k), dtype=torch.int64, device="cuda")
        ws = torch.empty(gpm.motif_enum_workspace_bytes(g, k), dtype=torch.uint8, device="cuda")
        out = torch.zeros_like(eager)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            gpm.motif_count_enum(g, k, ws=ws, out=out)   # warm up outside capture
        torch.cuda.current_stream().wait_stream(s)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            gpm.motif_count_enum(g, k, ws=ws, out=out)
        for r in range(4):
            out.zero_()
            junk = torch.randn(1000, device="cuda").sum()   # eager work between replays
            graph.replay()
            torch.cuda.synchronize()
            assert torch.equal(out, eager), (k, r)
            del junk


def test_5_motifs_above_map_limit(gpm):
    """A sparse graph above the map's vertex limit (binary searches): the 21
    5-motif counts equal the oracle's class by class."""
    e = graphgen.erdos_renyi(20000, 3.0 / 20000, 31)
    g = build(gpm, e)
    off, adj = oracle.canonical_csr(e.n, e.u, e.v)
    want = [oracle.pattern_count(off, adj, 5, gpm.motif_class_pattern(5, i), True)[0]
            for i in range(21)]
    assert sum(want) > 0
    assert gpm.motif_count_enum(g, 5) == want
