"""The general plan's matching order and symmetry-breaking partial orders
(host side, no GPU): every step after the first is adjacent to an earlier
one and wins Appendix B.3's greedy (more internal partial orders, then more
edges); the partial orders accept exactly one of the |Aut(P)| maps of any
embedding, checked over every labelling of the pattern's vertices."""
import itertools

import pytest

import paper_2011_03135_amd as gpm


def automorphisms(k, edges):
    E = {frozenset(e) for e in edges}
    out = []
    for p in itertools.permutations(range(k)):
        if all(frozenset((p[a], p[b])) in E for a, b in edges):
            out.append(p)
    return out


def connected_patterns(k):
    """All connected graphs on k vertices up to isomorphism (k <= 5)."""
    pairs = list(itertools.combinations(range(k), 2))
    seen, out = set(), []
    for mask in range(1, 1 << len(pairs)):
        edges = [pairs[i] for i in range(len(pairs)) if (mask >> i) & 1]
        if len(edges) < k - 1:
            continue
        adj = {v: set() for v in range(k)}
        for a, b in edges:
            adj[a].add(b)
            adj[b].add(a)
        stack, reach = [0], {0}
        while stack:
            x = stack.pop()
            for y in adj[x] - reach:
                reach.add(y)
                stack.append(y)
        if len(reach) < k:
            continue
        canon = min(tuple(sorted(tuple(sorted((p[a], p[b]))) for a, b in edges))
                    for p in itertools.permutations(range(k)))
        if canon not in seen:
            seen.add(canon)
            out.append(edges)
    return out


PATTERNS = [(k, e) for k in (3, 4, 5) for e in connected_patterns(k)
            if len(e) < k * (k - 1) // 2]           # cliques take the DAG plan
PATTERNS += [(6, [(i, i + 1) for i in range(5)]),                       # 6-path
             (6, [(i, (i + 1) % 6) for i in range(6)]),                  # 6-cycle
             (6, [(0, i) for i in range(1, 6)]),                         # 5-star
             (6, [(0, 1), (1, 2), (2, 0), (3, 4), (4, 5), (5, 3), (0, 3)])]  # two triangles


def test_pattern_census():
    # 2 connected 3-vertex graphs, 6 of 4, 21 of 5 (cliques excluded above)
    assert [len(connected_patterns(k)) for k in (3, 4, 5)] == [2, 6, 21]


@pytest.mark.parametrize("k,edges", PATTERNS)
@pytest.mark.parametrize("flags", [gpm.VERTEX_INDUCED, gpm.EDGE_INDUCED])
def test_matching_order_and_partial_orders(k, edges, flags):
    import ctypes
    p = gpm.pattern(k, edges, flags)
    plan = ctypes.c_int32()
    assert gpm.binding.load().gpm_pattern_plan(ctypes.byref(p), ctypes.byref(plan)) == 0
    if plan.value != 4:
        # the edge-induced diamond and 4-cycle take the subgraph-listing plans
        assert flags == gpm.EDGE_INDUCED and k == 4 and plan.value in (2, 3)
        return
    order, less = gpm.matching_order(p)
    assert sorted(order) == list(range(k))
    adj = {v: set() for v in range(k)}
    for a, b in edges:
        adj[a].add(b)
        adj[b].add(a)
    po = lambda x, y: int(y in less[x]) + int(x in less[y])   # noqa: E731
    # steps after the first: adjacent to an earlier one, and the greedy's choice
    for s in range(1, k):
        placed = order[:s]
        assert adj[order[s]] & set(placed), (order, s)
        if s >= 2:
            def score(x):
                return (sum(po(x, t) for t in placed), sum(1 for t in placed if t in adj[x]))
            cands = [x for x in range(k) if x not in placed and adj[x] & set(placed)]
            assert score(order[s]) == max(score(x) for x in cands), (order, s)
    # the first two steps carry a partial order whenever some edge does
    if any(po(a, b) for a, b in edges):
        assert po(order[0], order[1]) == 1
    # symmetry breaking: for every labelling f of the pattern's vertices,
    # exactly one automorphism sigma makes f o sigma satisfy the orders
    aut = automorphisms(k, edges)
    pairs = [(x, y) for x in range(k) for y in less[x]]
    for f in itertools.permutations(range(k)):
        ok = 0
        for sg in aut:
            g = [f[sg[x]] for x in range(k)]
            if all(g[x] < g[y] for x, y in pairs):
                ok += 1
        assert ok == 1, (edges, f)


def test_diamond_matches_triangle_first():
    """Appendix B.3's example: the vertex-induced diamond is matched
    triangle first, starting with the diagonal, whose two ends carry the
    partial order."""
    d = gpm.diamond(gpm.VERTEX_INDUCED)   # diagonal (0, 1), tips 2, 3
    order, less = gpm.matching_order(d)
    assert set(order[:2]) == {0, 1}
    assert (1 in less[0]) or (0 in less[1])
    assert order[2] in (2, 3)


def test_matching_order_other_plans_rejected():
    from paper_2011_03135_amd.binding import GpmError
    with pytest.raises(GpmError):
        gpm.matching_order(gpm.clique(4))
    with pytest.raises(GpmError):
        gpm.matching_order(gpm.cycle4())   # edge-induced: the subgraph-listing plan
