"""Closed forms the 5-motif formula route takes from the rows of A^2.  The
5-cycle count from closed walks (Harary and Manvel, 1971): a closed walk of
length 5 either runs once around a 5-cycle (ten such walks per cycle: five
starts, two directions) or goes around a triangle with one edge walked back
and forth, so

    N(C5) = [tr(A^5) - 5 tr(A^3) - 5 sum_v (d_v - 2) (A^3)_vv] / 10,

and with (A^3)_vv = 2 t_v, tr(A^3) = 6 T this is
[tr(A^5) - 30 T - 10 sum_v (d_v - 2) t_v] / 10.  Checked here, on the CPU,
against brute force over 5-vertex subsets and against the oracle's
edge-induced pattern count, on graphs whose 5-cycle counts are also known
in closed form.  And K_{2,3}: the sum over vertex pairs of C(common
neighbours, 3); the class of two non-adjacent vertices joined to an edge
and a fifth vertex, from pairs and triangles; K5 minus an edge, from
the vertices adjacent to all of a triangle; and the wheel, from the
4-cycles in each vertex's neighbourhood."""
from itertools import combinations, permutations

import numpy as np
import pytest

import brute
import graphgen
import oracle

C5 = [(0, 1), (1, 2), (2, 3), (3, 4), (4, 0)]


def formula_c5(n, u, v):
    A = np.zeros((n, n), dtype=np.int64)
    for a, b in zip(u, v):
        if a != b:
            A[a, b] = A[b, a] = 1
    A3 = A @ A @ A
    A5 = A3 @ A @ A
    d = A.sum(axis=1)
    t = np.diag(A3) // 2
    T = int(np.trace(A3)) // 6
    num = int(np.trace(A5)) - 30 * T - 10 * int(((d - 2) * t).sum())
    assert num % 10 == 0
    return num // 10


def brute_c5(n, u, v):
    adj = brute.adjacency_sets(n, u, v)
    count = 0
    for s in combinations(range(n), 5):
        a = s[0]
        # 5-cycles on the set s with a fixed first vertex and direction
        for p in permutations(s[1:]):
            if p[0] > p[3]:
                continue
            cyc = (a,) + p
            if all(cyc[(i + 1) % 5] in adj[cyc[i]] for i in range(5)):
                count += 1
    return count


def petersen():
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    e = outer + spokes + inner
    return graphgen.EdgeList(10, np.array([a for a, _ in e], np.int32),
                             np.array([b for _, b in e], np.int32), "petersen")


@pytest.mark.parametrize("case,closed", [
    ("k5", 12),          # (5 - 1)! / 2
    ("k6", 72),          # C(6, 5) * 12
    ("petersen", 12),
    ("c5", 1),
    ("k33", 0),          # bipartite: no odd cycle
    ("er12", None),
    ("er14", None),
    ("rmat6", None),
])
def test_five_cycle_closed_walk_formula(case, closed):
    e = {"k5": lambda: graphgen.complete_graph(5),
         "k6": lambda: graphgen.complete_graph(6),
         "petersen": petersen,
         "c5": lambda: graphgen.cycle_graph(5),
         "k33": lambda: graphgen.complete_bipartite(3, 3),
         "er12": lambda: graphgen.erdos_renyi(12, 0.5, 5),
         "er14": lambda: graphgen.erdos_renyi(14, 0.4, 6),
         "rmat6": lambda: graphgen.rmat(6, edge_factor=4, seed=6)}[case]()
    f = formula_c5(e.n, e.u, e.v)
    off, adj = oracle.canonical_csr(e.n, e.u, e.v)
    assert f == oracle.pattern_count(off, adj, 5, C5, induced=False)[0]
    if e.n <= 14:
        assert f == brute_c5(e.n, e.u, e.v)
    if closed is not None:
        assert f == closed


K23 = [(0, 2), (0, 3), (0, 4), (1, 2), (1, 3), (1, 4)]


def formula_k23(n, u, v):
    """K_{2,3} edge sets: a pair of vertices (the degree-3 side) and three of
    their common neighbours, so the sum over pairs of C(common, 3)."""
    from math import comb
    A = np.zeros((n, n), dtype=np.int64)
    for a, b in zip(u, v):
        if a != b:
            A[a, b] = A[b, a] = 1
    A2 = A @ A
    iu = np.triu_indices(n, 1)
    return sum(comb(int(c), 3) for c in A2[iu])


@pytest.mark.parametrize("case,closed", [
    ("k5", 10),          # C(5, 2) pairs, the other three vertices
    ("k33", 6),          # a pair on one side, the whole other side
    ("k28", 56),         # the pair of the 2-side, C(8, 3)
    ("petersen", 0),     # two vertices share at most one neighbour
    ("er14", None),
    ("rmat6", None),
])
def test_k23_pair_formula(case, closed):
    e = {"k5": lambda: graphgen.complete_graph(5),
         "k33": lambda: graphgen.complete_bipartite(3, 3),
         "k28": lambda: graphgen.complete_bipartite(2, 8),
         "petersen": petersen,
         "er14": lambda: graphgen.erdos_renyi(14, 0.4, 6),
         "rmat6": lambda: graphgen.rmat(6, edge_factor=4, seed=6)}[case]()
    f = formula_k23(e.n, e.u, e.v)
    off, adj = oracle.canonical_csr(e.n, e.u, e.v)
    assert f == oracle.pattern_count(off, adj, 5, K23, induced=False)[0]
    if closed is not None:
        assert f == closed


TWIN = [(0, 2), (1, 2), (0, 3), (1, 3), (2, 3), (0, 4), (1, 4)]   # class 16


def formula_twin(n, u, v):
    """Two non-adjacent vertices c, d joined to a, b, e with a ~ b: the pair
    {c, d} is unique, so N = sum over pairs of E_cd (k_cd - 2), with k_cd
    their common neighbours and E_cd the edges among them; that is S / 2 -
    2 D, S the sum over triangles {c, a, b} and common neighbours d != c of
    a and b of k_cd, and D the sum over edges of C(T_e, 2)."""
    from math import comb
    A = np.zeros((n, n), dtype=np.int64)
    for a, b in zip(u, v):
        if a != b:
            A[a, b] = A[b, a] = 1
    P2 = A @ A
    S = 0
    for c in range(n):
        nc = np.nonzero(A[c])[0]
        for ia in range(len(nc)):
            for ib in range(ia + 1, len(nc)):
                a, b = nc[ia], nc[ib]
                if A[a, b]:
                    S += int(sum(P2[c, d] for d in np.nonzero(A[a] & A[b])[0] if d != c))
    D = sum(comb(int(P2[a, b]), 2) for a in range(n) for b in range(a + 1, n) if A[a, b])
    assert S % 2 == 0
    return S // 2 - 2 * D


@pytest.mark.parametrize("case,closed", [
    ("k5", 30),          # 10 pairs {c, d}, 3 edges among the other three, 1 choice of e
    ("k33", 0),          # no edge among two vertices' common neighbours
    ("er12", None),
    ("er15", None),
    ("rmat6", None),
])
def test_twin_pair_formula(case, closed):
    e = {"k5": lambda: graphgen.complete_graph(5),
         "k33": lambda: graphgen.complete_bipartite(3, 3),
         "er12": lambda: graphgen.erdos_renyi(12, 0.5, 5),
         "er15": lambda: graphgen.erdos_renyi(15, 0.45, 7),
         "rmat6": lambda: graphgen.rmat(6, edge_factor=4, seed=6)}[case]()
    f = formula_twin(e.n, e.u, e.v)
    off, adj = oracle.canonical_csr(e.n, e.u, e.v)
    assert f == oracle.pattern_count(off, adj, 5, TWIN, induced=False)[0]
    if closed is not None:
        assert f == closed


K5E = [(0, 1), (0, 2), (1, 2), (0, 3), (1, 3), (2, 3), (0, 4), (1, 4), (2, 4)]


def formula_k5e(n, u, v):
    """K5 minus an edge: a triangle t (its degree-4 vertices) and two
    vertices adjacent to all of t, so the sum over triangles of C(k4(t), 2),
    k4(t) = the vertices adjacent to all of t; taken over each triangle at
    each of its three vertices, then divided by 3, as the kernel does."""
    from math import comb
    A = np.zeros((n, n), dtype=np.int64)
    for a, b in zip(u, v):
        if a != b:
            A[a, b] = A[b, a] = 1
    s = 0
    for c in range(n):
        nc = np.nonzero(A[c])[0]
        for ia in range(len(nc)):
            for ib in range(ia + 1, len(nc)):
                a, b = nc[ia], nc[ib]
                if A[a, b]:
                    s += comb(int((A[a] & A[b] & A[c]).sum()), 2)
    assert s % 3 == 0
    return s // 3


@pytest.mark.parametrize("case,closed", [
    ("k5", 10),          # C(5, 3) triangles, one pair of the other two each
    ("k6", 60),          # C(6, 3) triangles, C(3, 2) pairs each
    ("k33", 0),
    ("er12", None),
    ("er15", None),
    ("rmat6", None),
])
def test_k5e_triangle_formula(case, closed):
    e = {"k5": lambda: graphgen.complete_graph(5),
         "k6": lambda: graphgen.complete_graph(6),
         "k33": lambda: graphgen.complete_bipartite(3, 3),
         "er12": lambda: graphgen.erdos_renyi(12, 0.6, 5),
         "er15": lambda: graphgen.erdos_renyi(15, 0.5, 7),
         "rmat6": lambda: graphgen.rmat(6, edge_factor=4, seed=6)}[case]()
    f = formula_k5e(e.n, e.u, e.v)
    off, adj = oracle.canonical_csr(e.n, e.u, e.v)
    assert f == oracle.pattern_count(off, adj, 5, K5E, induced=False)[0]
    if closed is not None:
        assert f == closed


WHEEL = [(0, 1), (1, 2), (2, 3), (3, 0), (0, 4), (1, 4), (2, 4), (3, 4)]


def formula_wheel(n, u, v):
    """The wheel (a hub joined to all four vertices of a 4-cycle): its hub
    is its one vertex of degree 4, so the copies are the pairs (hub i,
    4-cycle in G[N(i)]).  A 4-cycle x-p-y-q is taken at its largest vertex x
    with y the vertex opposite x: for each x in N(i) and each y < x in N(i),
    C(c(x, y), 2) with c(x, y) the common neighbours p < x of x and y inside
    N(i), counted the way the kernel does, each increment of c adding the
    count before it."""
    A = np.zeros((n, n), dtype=np.int64)
    for a, b in zip(u, v):
        if a != b:
            A[a, b] = A[b, a] = 1
    total = 0
    for i in range(n):
        ni = set(np.nonzero(A[i])[0].tolist())
        for x in sorted(ni):
            cnt = {}
            for p in np.nonzero(A[x])[0]:
                if p >= x or p not in ni:
                    continue
                for y in np.nonzero(A[p])[0]:
                    if y < x and y in ni:
                        c = cnt.get(y, 0)
                        total += c
                        cnt[y] = c + 1
    return total


def wheel_graph(rim):
    pairs = [(i, (i + 1) % rim) for i in range(rim)] + [(i, rim) for i in range(rim)]
    return graphgen.graphs._as_edges(rim + 1, pairs, f"W{rim}")


@pytest.mark.parametrize("case,closed", [
    ("w4", 1),           # the pattern itself
    ("w5", 0),           # a 5-rim: no 4-cycle around any vertex
    ("k5", 15),          # 5 hubs, three 4-cycles in each K4
    ("k6", 90),          # 6 hubs, fifteen 4-cycles in each K5
    ("k2_2_2", 6),       # octahedron: each vertex's neighbourhood is one 4-cycle
    ("k33", 0),
    ("er12", None),
    ("er15", None),
    ("rmat6", None),
])
def test_wheel_neighbourhood_cycle_formula(case, closed):
    e = {"w4": lambda: wheel_graph(4),
         "w5": lambda: wheel_graph(5),
         "k5": lambda: graphgen.complete_graph(5),
         "k6": lambda: graphgen.complete_graph(6),
         "k2_2_2": lambda: graphgen.complete_multipartite([2, 2, 2]),
         "k33": lambda: graphgen.complete_bipartite(3, 3),
         "er12": lambda: graphgen.erdos_renyi(12, 0.6, 5),
         "er15": lambda: graphgen.erdos_renyi(15, 0.5, 7),
         "rmat6": lambda: graphgen.rmat(6, edge_factor=4, seed=6)}[case]()
    f = formula_wheel(e.n, e.u, e.v)
    off, adj = oracle.canonical_csr(e.n, e.u, e.v)
    assert f == oracle.pattern_count(off, adj, 5, WHEEL, induced=False)[0]
    if closed is not None:
        assert f == closed
