"""Pins of the CPU oracle against facts other than itself.

Each oracle function is checked against brute force over all vertex subsets
on tiny graphs (tests/brute.py, isomorphism by permutation), against closed
forms on structured graphs, against a library matrix product on the
Erdos-Renyi workload, and against the paper's worked local-counting example.
"""
import json
import math
import os
from itertools import combinations

import numpy as np
import pytest
import scipy.sparse as sp

import graphgen
import oracle
from oracle import canonical_csr
import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def csr(g):
    return canonical_csr(g.n, g.u, g.v)


def random_tiny(seed, n, p):
    g = graphgen.erdos_renyi(n, p, seed)
    return g


TINY = [(s, n, p) for s in range(1, 7) for n in (5, 8, 11) for p in (0.2, 0.45, 0.7, 0.9)]


@pytest.mark.parametrize("seed,n,p", TINY)
def test_brute_force_motifs_cliques(seed, n, p):
    g = random_tiny(seed, n, p)
    off, adj = csr(g)
    A = brute.adjacency_sets(g.n, g.u, g.v)
    m3 = brute.motif_counts(A, 3)
    assert oracle.motif3(off, adj) == [m3["wedge"], m3["triangle"]]
    m4 = brute.motif_counts(A, 4)
    assert oracle.motif4(off, adj) == [m4[k] for k in oracle.MOTIF4_NAMES]
    for k in (3, 4, 5):
        assert oracle.clique_count(off, adj, k) == brute.clique_count(A, k)


def _hash(codes):
    """The listing checksum's per-embedding hash, written out in Python."""
    M = (1 << 64) - 1

    def fin(z):
        z ^= z >> 30
        z = (z * 0xBF58476D1CE4E5B9) & M
        z ^= z >> 27
        z = (z * 0x94D049BB133111EB) & M
        z ^= z >> 31
        return z
    h = len(codes)
    for c in sorted(codes):
        h = fin(((h ^ c) + 0x9E3779B97F4A7C15) & M)
    return h


def _ecode(a, b):
    a, b = min(a, b), max(a, b)
    return (a << 32) | b


@pytest.mark.parametrize("seed,n,p", TINY[::3])
def test_brute_force_listings(seed, n, p):
    g = random_tiny(seed, n, p)
    off, adj = csr(g)
    A = brute.adjacency_sets(g.n, g.u, g.v)
    for name, fn, pat in (("diamond", oracle.list_diamonds, brute.PATTERNS4["diamond"]),
                          ("4-cycle", oracle.list_c4, brute.PATTERNS4["4-cycle"])):
        want = brute.edge_induced_embeddings(A, pat)
        total, chk, rows = fn(off, adj, cap=10 ** 6)
        assert total == len(want), name
        assert chk == sum(_hash([_ecode(a, b) for a, b in F]) for F in want) % (1 << 64)
        got = set()
        for r in rows.tolist():
            if name == "diamond":
                a, b, c, d = r
                F = [(a, b), (a, c), (a, d), (b, c), (b, d)]
            else:
                F = [(r[0], r[1]), (r[1], r[2]), (r[2], r[3]), (r[3], r[0])]
            got.add(frozenset(tuple(sorted(e)) for e in F))
        assert got == want
    for k in (3, 4):
        want = brute.clique_sets(A, k)
        total, chk, rows = oracle.clique_list(off, adj, k, cap=10 ** 6)
        assert total == len(want)
        assert {tuple(sorted(r)) for r in rows.tolist()} == want
        assert chk == sum(_hash(list(c)) for c in want) % (1 << 64)


def test_listing_truncation_keeps_total_and_checksum():
    g = graphgen.complete_graph(9)
    off, adj = csr(g)
    t_all, c_all, rows_all = oracle.list_diamonds(off, adj, cap=10 ** 5)
    t, c, rows = oracle.list_diamonds(off, adj, cap=7)
    assert (t, c) == (t_all, c_all) and rows.shape == (7, 4)


def C(a, b):
    return math.comb(a, b) if a >= b >= 0 else 0


@pytest.mark.parametrize("n", [1, 2, 3, 4, 7, 12])
def test_complete_graph(n):
    off, adj = csr(graphgen.complete_graph(n))
    for k in range(1, 8):
        assert oracle.clique_count(off, adj, k) == C(n, k)
    assert oracle.motif3(off, adj) == [0, C(n, 3)]
    assert oracle.motif4(off, adj) == [0, 0, 0, 0, 0, C(n, 4)]
    assert oracle.list_diamonds(off, adj)[0] == 6 * C(n, 4)
    assert oracle.list_c4(off, adj)[0] == 3 * C(n, 4)


def esym(parts, k):
    """Elementary symmetric polynomial e_k of the part sizes: a k-clique of a
    complete multipartite graph takes one vertex from each of k parts."""
    return sum(math.prod(c) for c in combinations(parts, k))


@pytest.mark.parametrize("parts", [[1, 2, 3], [2, 2, 2, 2], [5, 1, 4, 3, 2], [7, 7], [3, 9, 1, 1, 6]])
def test_complete_multipartite_cliques(parts):
    off, adj = csr(graphgen.complete_multipartite(parts))
    for k in range(2, 7):
        assert oracle.clique_count(off, adj, k) == esym(parts, k)


@pytest.mark.parametrize("leaves", [1, 2, 3, 6, 40])
def test_star(leaves):
    off, adj = csr(graphgen.star_graph(leaves))
    assert oracle.motif3(off, adj) == [C(leaves, 2), 0]
    assert oracle.motif4(off, adj) == [C(leaves, 3), 0, 0, 0, 0, 0]


@pytest.mark.parametrize("n", [4, 5, 6, 13])
def test_cycle(n):
    off, adj = csr(graphgen.cycle_graph(n))
    assert oracle.motif3(off, adj) == [n, 0]
    want = [0, 0, 1, 0, 0, 0] if n == 4 else [0, n, 0, 0, 0, 0]
    assert oracle.motif4(off, adj) == want


@pytest.mark.parametrize("a,b", [(1, 1), (2, 3), (3, 3), (4, 7)])
def test_complete_bipartite(a, b):
    off, adj = csr(graphgen.complete_bipartite(a, b))
    assert oracle.motif3(off, adj) == [a * C(b, 2) + b * C(a, 2), 0]
    assert oracle.motif4(off, adj) == [a * C(b, 3) + b * C(a, 3), 0, C(a, 2) * C(b, 2), 0, 0, 0]
    assert oracle.list_c4(off, adj)[0] == C(a, 2) * C(b, 2)


def _adj_matrix(off, adj):
    n = off.shape[0] - 1
    rows = np.repeat(np.arange(n), np.diff(off))
    return sp.csr_matrix((np.ones(adj.shape[0], dtype=np.int64), (rows, adj)), shape=(n, n))


def test_er_workload_trace_formulas():
    """The Erdos-Renyi workload G(4096, 0.004), seed 1: triangles equal
    trace(A^3)/6 and edge-induced 4-cycles equal (tr A^4 - 2 sum d^2 + sum d)/8
    (closed walks of length 4 minus the degenerate ones), by sparse library
    products in exact integers."""
    g = graphgen.erdos_renyi(4096, 0.004, 1)
    off, adj = csr(g)
    A = _adj_matrix(off, adj)
    A2 = A @ A
    tr3 = int(A2.multiply(A).sum())
    assert tr3 % 6 == 0
    assert oracle.triangle_count(off, adj) == tr3 // 6
    tr4 = int(A2.multiply(A2).sum())
    d = np.diff(off).astype(np.int64)
    c4 = tr4 - 2 * int((d * d).sum()) + int(d.sum())
    assert c4 % 8 == 0
    assert oracle.list_c4(off, adj)[0] == c4 // 8
    # edge-induced diamonds: pairs of triangles sharing an edge (Section 5)
    T = A2.multiply(A).data
    assert oracle.list_diamonds(off, adj)[0] == int((T * (T - 1) // 2).sum()) // 2


def test_paper_local_count_example():
    """Local-counting figure: an edge with 2 triangles whose ends have degree
    4 and 5 lies on 3 wedges.  Build such a graph and count by brute force."""
    with open(os.path.join(GOLDEN, "formula_example.json")) as f:
        ex = json.load(f)
    # u=0, v=1; common neighbours 2, 3; u's extra neighbour 4; v's extra 5, 6
    pairs = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (0, 4), (1, 5), (1, 6)]
    g = graphgen.EdgeList(7, np.array([p[0] for p in pairs], np.int32),
                          np.array([p[1] for p in pairs], np.int32))
    off, adj = csr(g)
    assert int(off[1] - off[0]) == ex["deg_u"] and int(off[2] - off[1]) == ex["deg_v"]
    te = oracle.edge_triangles(off, adj)
    e01 = int(off[0]) + int(np.searchsorted(adj[off[0]:off[1]], 1))
    assert te[e01] == ex["C_tri"]
    A = brute.adjacency_sets(g.n, g.u, g.v)
    wedges_on_e = sum(1 for w in range(g.n) if w not in (0, 1) and ((w in A[0]) != (w in A[1])))
    assert wedges_on_e == ex["C_wdg"]
    assert (ex["deg_u"] - ex["C_tri"] - 1) + (ex["deg_v"] - ex["C_tri"] - 1) == ex["C_wdg"]


def test_relabel_and_union_invariance():
    g = graphgen.erdos_renyi(60, 0.2, 5)
    h = graphgen.erdos_renyi(45, 0.3, 6)
    off, adj = csr(g)
    off2, adj2 = csr(graphgen.relabel(g, 9))
    assert oracle.motif4(off, adj) == oracle.motif4(off2, adj2)
    assert oracle.list_c4(off, adj)[0] == oracle.list_c4(off2, adj2)[0]
    offh, adjh = csr(h)
    offu, adju = csr(graphgen.disjoint_union([g, h]))
    for k in (3, 4, 5):
        assert oracle.clique_count(offu, adju, k) == \
            oracle.clique_count(off, adj, k) + oracle.clique_count(offh, adjh, k)
    a = oracle.motif4(off, adj)
    b = oracle.motif4(offh, adjh)
    assert oracle.motif4(offu, adju) == [x + y for x, y in zip(a, b)]


def test_canonical_csr_rules():
    u = np.array([3, 1, 1, 2, 2, 0, 3], np.int32)
    v = np.array([1, 3, 1, 0, 0, 2, 3], np.int32)
    off, adj = canonical_csr(4, u, v)
    assert off.tolist() == [0, 1, 2, 3, 4]
    rows = {x: adj[off[x]:off[x + 1]].tolist() for x in range(4)}
    assert rows == {0: [2], 1: [3], 2: [0], 3: [1]}
    with pytest.raises(ValueError):
        canonical_csr(4, np.array([0]), np.array([4]))


# ------------------------------------------- any connected pattern ---------

PATTERN_TINY = [(s, n, p) for s in (1, 2, 3) for n in (6, 8) for p in (0.35, 0.7)]


@pytest.mark.parametrize("seed,n,p", PATTERN_TINY)
@pytest.mark.parametrize("induced", [False, True])
def test_pattern_count_brute_force(seed, n, p, induced):
    g = random_tiny(seed, n, p)
    off, adj = csr(g)
    sets = brute.adjacency_sets(g.n, g.u, g.v)
    for name, (k, edges) in brute.PATTERNS_ANY.items():
        got, _ = oracle.pattern_count(off, adj, k, edges, induced)
        assert got == brute.pattern_embeddings(sets, k, edges, induced), (name, induced)


def test_pattern_count_closed_forms():
    off, adj = csr(graphgen.complete_graph(9))
    P = brute.PATTERNS_ANY
    for k in (3, 4, 5):
        name = {3: "triangle", 4: "4-clique", 5: "5-clique"}[k]
        assert oracle.pattern_count(off, adj, k, P[name][1], True)[0] == math.comb(9, k)
    # edge-induced 4-cycles in K_n: 3 per 4-set; 5-cycles: 12 per 5-set
    assert oracle.pattern_count(off, adj, 4, P["4-cycle"][1], False)[0] == 3 * math.comb(9, 4)
    assert oracle.pattern_count(off, adj, 5, P["5-cycle"][1], False)[0] == 12 * math.comb(9, 5)
    # any induced non-clique pattern is absent from a clique
    assert oracle.pattern_count(off, adj, 5, P["house"][1], True)[0] == 0
    # edge-induced stars and wedges: sum over centres of C(d, leaves)
    g = graphgen.erdos_renyi(120, 0.08, 5)
    off, adj = csr(g)
    deg = np.diff(off)
    assert oracle.pattern_count(off, adj, 3, P["wedge"][1], False)[0] == \
        sum(math.comb(int(x), 2) for x in deg)
    assert oracle.pattern_count(off, adj, 5, P["4-star"][1], False)[0] == \
        sum(math.comb(int(x), 4) for x in deg)
    # automorphism counts
    assert oracle.pattern_count(off, adj, 5, P["5-cycle"][1], False)[1] == 10
    assert oracle.pattern_count(off, adj, 5, P["house"][1], False)[1] == 2


def test_pattern_count_matches_other_routes():
    """Vertex-induced 4-patterns equal the 4-motif counts (back-substitution
    route); edge-induced diamond and 4-cycle equal the listing totals."""
    g = graphgen.erdos_renyi(70, 0.15, 9)
    off, adj = csr(g)
    want = oracle.motif4(off, adj)
    for i, name in enumerate(oracle.MOTIF4_NAMES):
        assert oracle.pattern_count(off, adj, 4, brute.PATTERNS4[name], True)[0] == want[i], name
    assert oracle.pattern_count(off, adj, 4, brute.PATTERNS4["diamond"], False)[0] == \
        oracle.list_diamonds(off, adj)[0]
    assert oracle.pattern_count(off, adj, 4, brute.PATTERNS4["4-cycle"], False)[0] == \
        oracle.list_c4(off, adj)[0]


# ------------------------------------------------------------ core numbers --
def brute_core_numbers(n, u, v):
    """The definition: the k-core is what remains after deleting vertices of
    degree < k until none is left; a vertex's core number is the largest k
    whose k-core holds it."""
    adj = brute.adjacency_sets(n, u, v)
    core = [0] * n
    k = 1
    alive = set(range(n))
    while alive:
        changed = True
        while changed:
            changed = False
            for x in list(alive):
                if sum(1 for y in adj[x] if y in alive) < k:
                    alive.discard(x)
                    changed = True
        for x in alive:
            core[x] = k
        k += 1
    return core


@pytest.mark.parametrize("seed", range(5))
def test_core_numbers_brute_force(seed):
    e = graphgen.erdos_renyi(40, 0.12 + 0.04 * seed, 300 + seed)
    off, adj = oracle.canonical_csr(e.n, e.u, e.v)
    assert list(oracle.core_numbers(off, adj)) == brute_core_numbers(e.n, e.u, e.v)


def test_core_numbers_closed_forms():
    cases = [(graphgen.complete_graph(9), lambda i: 8),
             (graphgen.star_graph(30), lambda i: 1),
             (graphgen.cycle_graph(25), lambda i: 2),
             (graphgen.path_graph(12), lambda i: 1),
             (graphgen.complete_bipartite(4, 9), lambda i: 4)]
    for e, want in cases:
        off, adj = oracle.canonical_csr(e.n, e.u, e.v)
        assert list(oracle.core_numbers(off, adj)) == [want(i) for i in range(e.n)], e.name
    # K_5 and a pendant path hanging off it: 4 on the clique, 1 on the path
    u = [a for a in range(5) for b in range(a + 1, 5)] + [4, 5, 6]
    v = [b for a in range(5) for b in range(a + 1, 5)] + [5, 6, 7]
    off, adj = oracle.canonical_csr(8, np.array(u, np.int32), np.array(v, np.int32))
    assert list(oracle.core_numbers(off, adj)) == [4, 4, 4, 4, 4, 1, 1, 1]


def brute_pattern_keys(A, k, edges, induced):
    """Every embedding of the pattern by brute force, as its canonical key:
    the vertex set (vertex-induced) or the edge set (edge-induced)."""
    target = brute.canon(k, edges)
    keys = set()
    for vs in combinations(range(len(A)), k):
        ind = brute.induced_edges(A, vs)
        if induced:
            if len(ind) == len(edges) and brute.canon(k, ind) == target:
                keys.add(tuple(vs))
            continue
        for F in combinations(ind, len(edges)):
            if len({x for e in F for x in e}) == k and brute.canon(k, list(F)) == target:
                keys.add(frozenset(tuple(sorted((vs[a], vs[b]))) for a, b in F))
    return keys


@pytest.mark.parametrize("seed,n,p", TINY[::4])
@pytest.mark.parametrize("induced", [False, True])
def test_pattern_list_brute_force(seed, n, p, induced):
    g = random_tiny(seed, n, p)
    off, adj = csr(g)
    A = brute.adjacency_sets(g.n, g.u, g.v)
    for name in ("wedge", "4-path", "4-cycle", "diamond", "house", "4-star"):
        k, edges = brute.PATTERNS_ANY[name]
        want = brute_pattern_keys(A, k, edges, induced)
        total, chk, rows = oracle.pattern_list(off, adj, k, edges, induced, cap=10 ** 6)
        assert total == len(want), name
        got = set()
        for r in rows.tolist():
            if induced:
                got.add(tuple(sorted(r)))
            else:
                got.add(frozenset(tuple(sorted((r[a], r[b]))) for a, b in edges))
        assert got == want, name
        if induced:
            assert chk == sum(_hash(list(key)) for key in want) % (1 << 64)
        else:
            assert chk == sum(_hash([_ecode(a, b) for a, b in key]) for key in want) % (1 << 64)
        assert total == oracle.pattern_count(off, adj, k, edges, induced)[0]


@pytest.mark.parametrize("n,k,stride", [(12, 3, 1), (12, 4, 5), (17, 5, 3), (9, 3, 9)])
def test_clique_count_sampled_complete_graph(n, k, stride):
    """In K_n the vertex at position p of any total order has n - 1 - p later
    neighbours, all adjacent, so the k-cliques it starts are C(n-1-p, k-1):
    each share of the roots has a closed form, whatever the order."""
    off, adj = csr(graphgen.complete_graph(n))
    dag = oracle.CoreDag(off, adj)
    for o in range(stride):
        want = sum(C(n - 1 - p, k - 1) for p in range(o, n, stride))
        assert oracle.clique_count_sampled(off, adj, k, stride, o) == want
        assert dag.clique_count_sampled(k, stride, o) == want
    dag.close()


@pytest.mark.parametrize("k", [3, 4, 5])
def test_clique_count_sampled_shares_add_up(k):
    """Every clique has exactly one first vertex, so the shares over all
    offsets add up to the clique count: on a complete multipartite graph
    (closed form e_k) and on an RMAT graph (the pinned clique count)."""
    parts = [3, 9, 1, 1, 6]
    off, adj = csr(graphgen.complete_multipartite(parts))
    assert sum(oracle.clique_count_sampled(off, adj, k, 4, o) for o in range(4)) == esym(parts, k)
    g = graphgen.rmat(12, seed=7)
    off, adj = csr(g)
    dag = oracle.CoreDag(off, adj)
    full = oracle.clique_count(off, adj, k)
    assert dag.clique_count_sampled(k, 1) == full
    shares = [dag.clique_count_sampled(k, 7, o) for o in range(7)]
    assert sum(shares) == full
    assert all(0 < s < full for s in shares)
    dag.close()
    with pytest.raises(RuntimeError):
        oracle.clique_count_sampled(off, adj, k, 7, 7)
