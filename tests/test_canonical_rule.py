"""The canonical-extension rule of the pattern-oblivious motif route, checked
by brute force: extending an embedding (v0, ..., v_{l-1}) by u only when
u > v0 and u exceeds every vertex after u's first neighbour in the
embedding reaches every connected vertex set of size k exactly once
(Appendix B.1: one embedding per automorphism class).  Pure Python; the
device kernel implements this rule as range cuts on sorted rows."""
from itertools import combinations
import random

import pytest

import brute


def canonical_sets(adj, k):
    seen = {}

    def extend(emb):
        if len(emb) == k:
            key = frozenset(emb)
            seen[key] = seen.get(key, 0) + 1
            return
        for i, vi in enumerate(emb):
            bound = max([emb[0]] + emb[i + 1:])
            for u in sorted(adj[vi]):
                if u <= bound or any(u in adj[emb[j]] for j in range(i)):
                    continue
                extend(emb + [u])

    for v in range(len(adj)):
        extend([v])
    return seen


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("k", [2, 3, 4, 5])
def test_each_connected_set_once(k, seed):
    rnd = random.Random(100 * k + seed)
    n, p = 13, 0.3
    pairs = [(a, b) for a in range(n) for b in range(a + 1, n) if rnd.random() < p]
    adj = brute.adjacency_sets(n, [a for a, _ in pairs], [b for _, b in pairs])
    seen = canonical_sets(adj, k)
    truth = {frozenset(vs) for vs in combinations(range(n), k)
             if brute.connected(k, brute.induced_edges(adj, vs))}
    assert set(seen) == truth
    assert all(c == 1 for c in seen.values())
