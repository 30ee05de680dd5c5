"""Roots of out-degree above 1024 (hub roots, too large for the LDS staging
of the triangle and local-graph kernels) are split at arc granularity and
mined by k_clique_hub, while every other root stays in its out-degree
class.  On a graph where over a thousand roots are hubs (the B side of a
complete bipartite K_{1030,1030}, and a vertex joined to all of A, with
random edges inside A) next to an RMAT graph, every count and listing
equals the oracle's."""
import numpy as np
import pytest

import graphgen
import oracle
from oracle import canonical_csr
from gpu_util import build

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpm():
    import paper_2011_03135_amd as m
    m.load()
    return m


def hub_graph(side=1030, p=0.04, seed=5):
    """A = [0, side), B = [side, 2 side), every A-B edge, the vertex 2 side
    joined to all of A, and each pair inside A an edge with probability p.
    Every B vertex and the extra vertex have all their neighbours above them
    in the degree order: out-degree `side`."""
    rng = np.random.default_rng(seed)
    A = np.arange(side)
    au, bu = np.meshgrid(A, np.arange(side, 2 * side), indexing="ij")
    iu, ju = np.triu_indices(side, 1)
    keep = rng.random(iu.shape[0]) < p
    u = np.concatenate([au.ravel(), np.full(side, 2 * side), iu[keep]]).astype(np.int32)
    v = np.concatenate([bu.ravel(), A, ju[keep]]).astype(np.int32)
    return graphgen.EdgeList(2 * side + 1, u, v, "hubs")


@pytest.fixture(scope="module")
def case(gpm):
    e = graphgen.disjoint_union([hub_graph(), graphgen.rmat(12, seed=12)])
    g = build(gpm, e)
    off, adj = canonical_csr(e.n, e.u, e.v)
    assert g.max_out_degree > 1024
    return e, g, off, adj


def test_hub_clique_counts(gpm, case):
    e, g, off, adj = case
    want = {k: oracle.clique_count(off, adj, k) for k in (3, 4, 5, 6)}
    for k in (3, 4, 5, 6):
        print(f"hub graph {k}-cliques", flush=True)
        assert gpm.count(g, gpm.clique(k)) == want[k], k
    assert gpm.clique_counts(g, 4) == [want[3], want[4]]
    assert gpm.clique_counts(g, 5) == [want[3], want[4], want[5]]


def test_hub_motifs_and_subgraph_counts(gpm, case):
    e, g, off, adj = case
    assert gpm.motif_count(g, 3) == oracle.motif3(off, adj)
    assert gpm.motif_count(g, 4) == oracle.motif4(off, adj)
    # edge-induced diamonds and 4-cycles are the non-induced copies
    n4 = oracle.motif4_noninduced(off, adj)
    assert gpm.count(g, gpm.diamond()) == n4[4]
    assert gpm.count(g, gpm.cycle4()) == n4[2]


@pytest.mark.parametrize("k", [3, 4, 5])
def test_hub_clique_listing(gpm, case, k):
    e, g, off, adj = case
    total, chk, _ = oracle.clique_list(off, adj, k, cap=0)
    cap = 1 << 20
    t, w, c, rows = gpm.list_embeddings(g, gpm.clique(k, gpm.VERTEX_INDUCED | gpm.LIST), cap)
    assert (t, w, c) == (total, min(total, cap), chk)
    # written rows are cliques of distinct vertices
    r = rows.cpu().numpy().astype(np.int64)
    n = off.shape[0] - 1
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(off))
    codes = np.sort(src * (1 << 32) + adj.astype(np.int64))
    for a in range(k):
        for b in range(a + 1, k):
            q = r[:, a] * (1 << 32) + r[:, b]
            pos = np.minimum(np.searchsorted(codes, q), codes.shape[0] - 1)
            assert np.all(codes[pos] == q)
    assert len({tuple(sorted(x)) for x in r.tolist()}) == r.shape[0]
