"""Induced 3- and 4-motif counts (local counting) against the CPU oracle."""
import json
import os

import numpy as np
import pytest

import graphgen
import oracle
from oracle import canonical_csr
from gpu_util import build

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "rmat_counts.json")


@pytest.fixture(scope="module")
def gpm():
    import paper_2011_03135_amd as m
    m.load()
    return m


def cases():
    return [
        graphgen.star_graph(30),
        graphgen.cycle_graph(4),
        graphgen.cycle_graph(9),
        graphgen.complete_bipartite(5, 8),
        graphgen.complete_graph(9),
        graphgen.path_graph(6),
        graphgen.erdos_renyi(120, 0.08, 21),
        graphgen.erdos_renyi(400, 0.03, 22),
        graphgen.rmat(11, seed=31),
        graphgen.rmat(14, seed=14),
        graphgen.star_graph(2000),                      # one heavy apex
        graphgen.complete_bipartite(40, 300),            # heavy apexes, many 4-cycles
        graphgen.EdgeList(3, np.zeros(0, np.int32), np.zeros(0, np.int32), "empty"),
    ]


@pytest.mark.parametrize("case", range(13))
def test_motif_counts(gpm, case):
    e = cases()[case]
    print(f"motif case {case} {e.name}", flush=True)
    g = build(gpm, e)
    off, adj = canonical_csr(e.n, e.u, e.v)
    assert gpm.motif_count(g, 3) == oracle.motif3(off, adj), e.name
    assert gpm.motif_count(g, 4) == oracle.motif4(off, adj), e.name


def test_motif_disjoint_union_additive(gpm):
    a = graphgen.erdos_renyi(90, 0.1, 3)
    b = graphgen.rmat(10, seed=4)
    ga, gb = build(gpm, a), build(gpm, b)
    gu = build(gpm, graphgen.disjoint_union([a, b]))
    for k in (3, 4):
        x, y, z = gpm.motif_count(ga, k), gpm.motif_count(gb, k), gpm.motif_count(gu, k)
        assert z == [p + q for p, q in zip(x, y)]


def test_rmat18_motifs_golden(gpm):
    if not os.path.exists(GOLDEN):
        pytest.skip("golden counts not generated")
    with open(GOLDEN) as f:
        gold = json.load(f).get("rmat18", {})
    if "motif4" not in gold:
        pytest.skip("rmat18 motif golden counts not generated")
    g = build(gpm, graphgen.rmat(18, seed=18))
    assert gpm.motif_count(g, 3) == gold["motif3"]
    assert gpm.motif_count(g, 4) == gold["motif4"]


def C(n, k):
    from math import comb
    return comb(n, k)


def test_four_cycle_counter_widths(gpm):
    """The 4-cycle counters are 16 bits when at most one vertex has a degree
    above 65535 (a star's centre of degree 70,000 next to K_{3,300}) and 32
    bits otherwise (K_{2,70000}: two such vertices, a counter reaching
    70,000); closed forms for both: K_{a,b} holds C(a,2) C(b,2) 4-cycles and
    a C(b,3) + b C(a,3) 3-stars."""
    star_k = graphgen.disjoint_union([graphgen.star_graph(70000),
                                      graphgen.complete_bipartite(3, 300)])
    g = build(gpm, star_k)
    c4 = C(3, 2) * C(300, 2)
    assert gpm.count(g, gpm.cycle4()) == c4
    claws = C(70000, 3) + 3 * C(300, 3) + 300 * C(3, 3)
    assert gpm.motif_count(g, 4) == [claws, 0, c4, 0, 0, 0]
    kb = graphgen.complete_bipartite(2, 70000)
    g = build(gpm, kb)
    c4 = C(2, 2) * C(70000, 2)
    assert gpm.count(g, gpm.cycle4()) == c4
    assert gpm.motif_count(g, 4) == [2 * C(70000, 3), 0, c4, 0, 0, 0]


def test_four_cycles_without_part_table(gpm):
    """A 5,000,000-vertex graph, too large for the heavy 4-cycle kernel's part
    table (parts x n x 8 B above 2 GiB), so each middle's segment of a z-part
    is found by binary search.  40 hubs joined to the same 300 middles and to
    1,000 leaves each, every middle with 300 leaves of its own, the rest
    isolated, ids scattered by a seeded permutation: the hubs' wedges end in
    other hubs and in 90,000 middles' leaves, whose low ranks spread over
    several parts.  The 4-cycles are those of K_{40,300}: C(40,2) C(300,2);
    all six 4-motif counts against the oracle."""
    n, hubs, mids, hub_leaves, mid_leaves = 5_000_000, 40, 300, 1000, 300
    h = np.arange(hubs, dtype=np.int64)
    m = hubs + np.arange(mids, dtype=np.int64)
    u = [np.repeat(h, mids)]
    v = [np.tile(m, hubs)]
    base = hubs + mids
    u.append(np.repeat(h, hub_leaves))
    v.append(base + np.arange(hubs * hub_leaves, dtype=np.int64))
    base += hubs * hub_leaves
    u.append(np.repeat(m, mid_leaves))
    v.append(base + np.arange(mids * mid_leaves, dtype=np.int64))
    e = graphgen.EdgeList(n, np.concatenate(u).astype(np.int32),
                          np.concatenate(v).astype(np.int32), "hubs_mids_leaves")
    e = graphgen.relabel(e, 7)
    print(f"four cycles without part table: n={e.n} m={e.u.shape[0]}", flush=True)
    g = build(gpm, e)
    assert gpm.count(g, gpm.cycle4()) == C(hubs, 2) * C(mids, 2)
    off, adj = canonical_csr(e.n, e.u, e.v)
    assert gpm.motif_count(g, 4) == oracle.motif4(off, adj)
