"""General connected patterns (2..6 vertices, vertex- or edge-induced)
counted on the device against the oracle's plain enumeration."""
import numpy as np
import pytest

import brute
import graphgen
import oracle
from gpu_util import build

pytestmark = pytest.mark.gpu

EXTRA = {
    "edge": (2, [(0, 1)]),
    "6-cycle": (6, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 5), (5, 0)]),
    "domino": (6, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 5), (5, 0), (1, 4)]),
    "6-path": (6, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 5)]),
    "tadpole": (6, [(0, 1), (1, 2), (2, 0), (2, 3), (3, 4), (4, 5)]),
}
PATTERNS = {**brute.PATTERNS_ANY, **EXTRA}


@pytest.fixture(scope="module")
def gpm():
    import paper_2011_03135_amd as m
    m.load()
    return m


def hub_graph():
    """ER(100, 0.06) plus a hub joined to 45 vertices: skewed degrees that
    the oracle's plain enumeration still finishes in seconds."""
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
            graphgen.star_graph(40)]


@pytest.mark.parametrize("gi", range(5))
@pytest.mark.parametrize("induced", [False, True])
def test_patterns_vs_oracle(gpm, gi, induced):
    e = graphs()[gi]
    print(f"graph {gi} n={e.n} induced={induced}", flush=True)
    g = build(gpm, e)
    off, adj = oracle.canonical_csr(e.n, e.u, e.v)
    flags = gpm.VERTEX_INDUCED if induced else gpm.EDGE_INDUCED
    for name, (k, edges) in PATTERNS.items():
        want, _ = oracle.pattern_count(off, adj, k, edges, induced)
        got = gpm.count(g, gpm.pattern(k, edges, flags))
        assert got == want, (name, induced)


def test_degree_filter_off_same_counts(gpm, monkeypatch):
    """Degree filtering (Section 4.3) only skips candidates that cannot
    match: with GPM_DF=0 every count, and a listing's total and checksum,
    are the same."""
    e = hub_graph()
    g = build(gpm, e)
    pats = [(name, PATTERNS[name]) for name in ("4-cycle", "4-path", "house", "5-cycle",
                                                   "domino", "tadpole")]
    want = {}
    for name, (k, edges) in pats:
        for flags in (gpm.EDGE_INDUCED, gpm.VERTEX_INDUCED):
            want[(name, flags)] = gpm.count(g, gpm.pattern(k, edges, flags))
    house = gpm.pattern(5, [(0, 1), (1, 2), (2, 3), (3, 0), (2, 4), (3, 4)],
                        gpm.EDGE_INDUCED | gpm.LIST)
    lw = gpm.list_embeddings(g, house, 1 << 16)[:3]
    monkeypatch.setenv("GPM_DF", "0")
    for name, (k, edges) in pats:
        for flags in (gpm.EDGE_INDUCED, gpm.VERTEX_INDUCED):
            assert gpm.count(g, gpm.pattern(k, edges, flags)) == want[(name, flags)], name
    house = gpm.pattern(5, [(0, 1), (1, 2), (2, 3), (3, 0), (2, 4), (3, 4)],
                        gpm.EDGE_INDUCED | gpm.LIST)
    assert gpm.list_embeddings(g, house, 1 << 16)[:3] == lw


def test_relabelled_pattern_same_count(gpm):
    """The same pattern under another vertex numbering (another matching
    order and other partial orders) gives the same count."""
    e = graphgen.erdos_renyi(120, 0.07, 4)
    g = build(gpm, e)
    house = [(0, 1), (1, 2), (2, 3), (3, 0), (2, 4), (3, 4)]
    perm = [3, 0, 4, 1, 2]
    relabel = [(perm[a], perm[b]) for a, b in house]
    for flags in (gpm.EDGE_INDUCED, gpm.VERTEX_INDUCED):
        assert gpm.count(g, gpm.pattern(5, house, flags)) == \
            gpm.count(g, gpm.pattern(5, relabel, flags))


def test_generic_closed_forms_rmat(gpm):
    """Properties that hold at any size: edge-induced wedges and 3-stars are
    sums of binomials of the degrees; vertex-induced 4-paths and 4-cycles
    equal the 4-motif counts of the local-count route."""
    e = graphgen.rmat(11, seed=7)
    g = build(gpm, e)
    off, adj = oracle.canonical_csr(e.n, e.u, e.v)
    deg = np.diff(off).astype(object)
    P = brute.PATTERNS_ANY
    assert gpm.count(g, gpm.pattern(3, P["wedge"][1], gpm.EDGE_INDUCED)) == \
        sum(d * (d - 1) // 2 for d in deg)
    assert gpm.count(g, gpm.pattern(4, P["3-star"][1], gpm.EDGE_INDUCED)) == \
        sum(d * (d - 1) * (d - 2) // 6 for d in deg)
    motifs = gpm.motif_count(g, 4)
    names = list(gpm.MOTIF4_NAMES)
    for name in ("4-path", "4-cycle", "tailed-triangle"):
        got = gpm.count(g, gpm.pattern(4, P[name][1], gpm.VERTEX_INDUCED))
        assert got == motifs[names.index(name)], name


def _keys(rows, edges, induced):
    if induced:
        return {tuple(sorted(r)) for r in rows}
    return {frozenset(tuple(sorted((r[a], r[b]))) for a, b in edges) for r in rows}


@pytest.mark.parametrize("gi", [0, 2])
@pytest.mark.parametrize("induced", [False, True])
def test_listing_vs_oracle(gpm, gi, induced):
    """Listing: the same embeddings (as canonical keys), total and checksum
    as the oracle's listing; a truncated listing keeps total and checksum
    and writes valid embeddings only."""
    e = graphs()[gi]
    print(f"graph {gi} n={e.n} induced={induced}", flush=True)
    g = build(gpm, e)
    off, adj = oracle.canonical_csr(e.n, e.u, e.v)
    flags = (gpm.VERTEX_INDUCED if induced else gpm.EDGE_INDUCED) | gpm.LIST
    for name in ("edge", "wedge", "4-path", "tailed-triangle", "house", "bull", "6-path"):
        k, edges = PATTERNS[name]
        full = 1 << 21
        total, chk, rows = oracle.pattern_list(off, adj, k, edges, induced, cap=full)
        t, w, c, got = gpm.list_embeddings(g, gpm.pattern(k, edges, flags), full)
        assert (t, w, c) == (total, min(total, full), chk), name
        if total <= full:
            assert _keys(got.cpu().tolist(), edges, induced) == \
                _keys(rows.tolist(), edges, induced), name
        cap = max(1, total // 3)
        t, w, c, got = gpm.list_embeddings(g, gpm.pattern(k, edges, flags), cap)
        assert (t, w, c) == (total, min(cap, total), chk), name
        if total <= full:
            assert _keys(got.cpu().tolist(), edges, induced) <= \
                _keys(rows.tolist(), edges, induced), name


def test_listing_without_map(gpm, monkeypatch):
    e = graphs()[0]
    g = build(gpm, e)
    off, adj = oracle.canonical_csr(e.n, e.u, e.v)
    monkeypatch.setenv("GPM_MNC", "0")
    k, edges = PATTERNS["house"]
    for induced in (False, True):
        flags = (gpm.VERTEX_INDUCED if induced else gpm.EDGE_INDUCED) | gpm.LIST
        total, chk, _ = oracle.pattern_list(off, adj, k, edges, induced, cap=0)
        t, w, c, _ = gpm.list_embeddings(g, gpm.pattern(k, edges, flags), 1 << 16)
        assert (t, c) == (total, chk)


def test_generic_errors(gpm):
    e = graphgen.erdos_renyi(30, 0.2, 5)
    g = build(gpm, e)
    with pytest.raises(gpm.GpmError):
        gpm.count(g, gpm.pattern(7, [(i, i + 1) for i in range(6)], gpm.EDGE_INDUCED))


@pytest.mark.parametrize("gi", [0, 2])
def test_without_connectivity_map(gpm, gi, monkeypatch):
    """GPM_MNC=0: adjacency from binary searches instead of the per-wave map
    (patterns of up to 5 vertices use the map by default)."""
    e = graphs()[gi]
    print(f"graph {gi} n={e.n}", flush=True)
    g = build(gpm, e)
    off, adj = oracle.canonical_csr(e.n, e.u, e.v)
    monkeypatch.setenv("GPM_MNC", "0")
    for induced in (False, True):
        flags = gpm.VERTEX_INDUCED if induced else gpm.EDGE_INDUCED
        for name, (k, edges) in PATTERNS.items():
            if k > 5:
                continue
            want, _ = oracle.pattern_count(off, adj, k, edges, induced)
            assert gpm.count(g, gpm.pattern(k, edges, flags)) == want, (name, induced)


def test_map_limit(gpm):
    """A graph above the map's vertex limit (binary searches) and the
    local-count route agree on the induced 4-cycles and 4-paths."""
    e = graphgen.erdos_renyi(20000, 8.0 / 20000, 12)
    g = build(gpm, e)
    motifs = gpm.motif_count(g, 4)
    names = list(gpm.MOTIF4_NAMES)
    P = brute.PATTERNS_ANY
    for name in ("4-path", "4-cycle"):
        got = gpm.count(g, gpm.pattern(4, P[name][1], gpm.VERTEX_INDUCED))
        assert got == motifs[names.index(name)], name
