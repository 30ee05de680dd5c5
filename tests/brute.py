"""Brute-force pattern mining for tiny graphs (pure Python; n up to ~14).

Independent of both the oracle and the device path: it enumerates every
vertex subset (or every edge subset of every 4-vertex set) and decides
isomorphism by trying all vertex permutations.
"""
from itertools import combinations, permutations


def adjacency_sets(n, u, v):
    adj = [set() for _ in range(n)]
    for a, b in zip(u, v):
        a, b = int(a), int(b)
        if a != b:
            adj[a].add(b)
            adj[b].add(a)
    return adj


def canon(k, edges):
    """Canonical form of a k-vertex graph: lexicographically least sorted
    edge list over all relabellings."""
    best = None
    for p in permutations(range(k)):
        e = sorted(tuple(sorted((p[a], p[b]))) for a, b in edges)
        if best is None or e < best:
            best = e
    return tuple(best)


def connected(k, edges):
    if k == 0:
        return True
    nb = [set() for _ in range(k)]
    for a, b in edges:
        nb[a].add(b)
        nb[b].add(a)
    seen, stack = {0}, [0]
    while stack:
        x = stack.pop()
        for y in nb[x]:
            if y not in seen:
                seen.add(y)
                stack.append(y)
    return len(seen) == k


# pattern edge lists on vertices 0..k-1
PATTERNS3 = {"wedge": [(0, 1), (1, 2)], "triangle": [(0, 1), (1, 2), (0, 2)]}
PATTERNS4 = {
    "3-star": [(0, 1), (0, 2), (0, 3)],
    "4-path": [(0, 1), (1, 2), (2, 3)],
    "4-cycle": [(0, 1), (1, 2), (2, 3), (3, 0)],
    "tailed-triangle": [(0, 1), (1, 2), (0, 2), (2, 3)],
    "diamond": [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3)],
    "4-clique": [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)],
}


def induced_edges(adj, vs):
    idx = {x: i for i, x in enumerate(vs)}
    return [(idx[a], idx[b]) for a, b in combinations(vs, 2) if b in adj[a]]


def motif_counts(adj, k):
    """Induced counts of every connected k-vertex pattern, by name."""
    pats = PATTERNS3 if k == 3 else PATTERNS4
    key = {canon(k, e): name for name, e in pats.items()}
    out = {name: 0 for name in pats}
    for vs in combinations(range(len(adj)), k):
        e = induced_edges(adj, vs)
        if not connected(k, e):
            continue
        out[key[canon(k, e)]] += 1
    return out


def clique_count(adj, k):
    return sum(1 for vs in combinations(range(len(adj)), k)
               if all(b in adj[a] for a, b in combinations(vs, 2)))


def edge_induced_embeddings(adj, pattern_edges):
    """Every distinct edge set F of the graph whose edge-induced subgraph is
    isomorphic to the pattern (4-vertex connected patterns): returns a set of
    frozensets of (min, max) edges."""
    k = 4
    target = canon(k, pattern_edges)
    ne = len(pattern_edges)
    found = set()
    for vs in combinations(range(len(adj)), k):
        ind = [(vs[a], vs[b]) for a, b in induced_edges(adj, vs)]
        idx = {x: i for i, x in enumerate(vs)}
        for F in combinations(ind, ne):
            local = [(idx[a], idx[b]) for a, b in F]
            touched = {x for e in local for x in e}
            if len(touched) != k:
                continue
            if canon(k, local) == target:
                found.add(frozenset(tuple(sorted(e)) for e in F))
    return found


def clique_sets(adj, k):
    return {vs for vs in combinations(range(len(adj)), k)
            if all(b in adj[a] for a, b in combinations(vs, 2))}


# connected patterns of 3..5 vertices for the general-pattern tests: (k, edges)
PATTERNS_ANY = {
    "wedge": (3, [(0, 1), (1, 2)]),
    "triangle": (3, [(0, 1), (1, 2), (0, 2)]),
    **{name: (4, e) for name, e in PATTERNS4.items()},
    "5-path": (5, [(0, 1), (1, 2), (2, 3), (3, 4)]),
    "4-star": (5, [(0, 1), (0, 2), (0, 3), (0, 4)]),
    "5-cycle": (5, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 0)]),
    "house": (5, [(0, 1), (1, 2), (2, 3), (3, 0), (2, 4), (3, 4)]),
    "bull": (5, [(0, 1), (1, 2), (0, 2), (1, 3), (2, 4)]),
    "gem": (5, [(0, 1), (0, 2), (0, 3), (0, 4), (1, 2), (2, 3), (3, 4)]),
    "5-clique": (5, [(a, b) for a in range(5) for b in range(a + 1, 5)]),
}


def pattern_embeddings(adj, k, pattern_edges, induced):
    """Number of embeddings of a connected k-vertex pattern: vertex-induced,
    the k-sets whose induced subgraph is isomorphic to it; edge-induced, the
    distinct edge sets F (spanning k vertices) isomorphic to it."""
    target = canon(k, pattern_edges)
    ne = len(pattern_edges)
    count = 0
    for vs in combinations(range(len(adj)), k):
        ind = induced_edges(adj, vs)
        if induced:
            count += len(ind) == ne and canon(k, ind) == target
            continue
        for F in combinations(ind, ne):
            if len({x for e in F for x in e}) == k and canon(k, list(F)) == target:
                count += 1
    return count
