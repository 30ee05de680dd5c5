"""Induced 5-motif counts by formulas (local counts, rows of A^2, the
4-cycles in each neighbourhood, the clique kernels for K5, the general plan
above the LDS limit, back-substitution) against the oracle class by class,
against closed forms, and against the enumeration route."""
from math import comb

import numpy as np
import pytest

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
    base = graphgen.erdos_renyi(90, 0.08, 5)
    rng = np.random.default_rng(5)
    ends = rng.choice(np.arange(1, 90), size=40, replace=False).astype(np.int32)
    return graphgen.EdgeList(90, np.concatenate([base.u, np.zeros(40, np.int32)]),
                             np.concatenate([base.v, ends]), "hub")


def cases():
    return [graphgen.erdos_renyi(40, 0.2, 1),
            graphgen.erdos_renyi(60, 0.12, 2),
            graphgen.rmat(8, seed=3),
            hub_graph(),
            graphgen.disjoint_union([graphgen.complete_graph(7), graphgen.cycle_graph(8),
                                     graphgen.star_graph(9)]),
            graphgen.EdgeList(6, np.zeros(0, np.int32), np.zeros(0, np.int32), "empty")]


@pytest.mark.parametrize("case", range(6))
def test_formula_route_vs_oracle(gpm, case):
    e = cases()[case]
    print(f"5-motif formula case {case} {e.name}", flush=True)
    g = build(gpm, e)
    off, adj = oracle.canonical_csr(e.n, e.u, e.v)
    want = [oracle.pattern_count(off, adj, 5, gpm.motif_class_pattern(5, i), True)[0]
            for i in range(21)]
    assert gpm.motif_count_formula(g, 5) == want


def test_formula_route_closed_forms(gpm):
    def only(i, v):
        out = [0] * 21
        out[i] = v
        return out
    assert gpm.motif_count_formula(build(gpm, graphgen.complete_graph(9)), 5) == only(20, comb(9, 5))
    assert gpm.motif_count_formula(build(gpm, graphgen.star_graph(30)), 5) == only(0, comb(30, 4))
    assert gpm.motif_count_formula(build(gpm, graphgen.cycle_graph(11)), 5) == only(2, 11)
    # K_{3,6}: 4-stars centred on the small side, K_{2,3} either way round
    want = [0] * 21
    want[0] = 3 * comb(6, 4)
    want[10] = comb(3, 2) * comb(6, 3) + comb(3, 3) * comb(6, 2)
    assert gpm.motif_count_formula(build(gpm, graphgen.complete_bipartite(3, 6)), 5) == want


@pytest.mark.parametrize("scale", [10, 12])
def test_formula_route_equals_enumeration(gpm, scale):
    """The two device routes, formulas and pattern-oblivious enumeration,
    give the same 21 counts on RMAT graphs."""
    g = build(gpm, graphgen.rmat(scale, seed=scale))
    print(f"rmat{scale} 5-motifs", flush=True)
    assert gpm.motif_count_formula(g, 5) == gpm.motif_count_enum(g, 5)


def test_formula_route_rejects(gpm):
    from paper_2011_03135_amd.binding import GpmError
    g = build(gpm, graphgen.erdos_renyi(30, 0.2, 3))
    with pytest.raises(GpmError):
        gpm.motif_count_formula(g, 4)


def test_formula_route_wide_counters(gpm):
    """Two vertices of degree above 65535 (two stars with adjacent centres)
    next to K_{3,300}: the 4-cycle counters and their cycle sums run with
    32-bit counters.  Closed forms: a centre with its neighbours gives the
    4-stars, a centre with two of its leaves and one of the other's gives
    the chairs, K_{3,300} adds 3 C(300, 4) 4-stars and 3 C(300, 3) + C(300, 2)
    copies of K_{2,3}."""
    a = b = 70000
    s1, s2 = graphgen.star_graph(a), graphgen.star_graph(b)
    kb = graphgen.complete_bipartite(3, 300)
    two = graphgen.disjoint_union([s1, s2, kb])
    # join the two centres (vertex 0 of each star)
    e = graphgen.EdgeList(two.n, np.concatenate([two.u, np.array([0], np.int32)]),
                          np.concatenate([two.v, np.array([s1.n], np.int32)]), "double_star")
    g = build(gpm, e)
    want = [0] * 21
    want[0] = comb(a + 1, 4) + comb(b + 1, 4) + 3 * comb(300, 4)
    want[1] = comb(a, 2) * b + comb(b, 2) * a
    want[10] = 3 * comb(300, 3) + comb(300, 2)
    assert gpm.motif_count_formula(g, 5) == want


def test_formula_route_core_orientation(gpm):
    """Under the core-value orientation (a different DAG: other triangle
    arcs, other 4-clique roots) the formula route gives the same counts."""
    g = build(gpm, graphgen.rmat(10, seed=10))
    want = gpm.motif_count_formula(g, 5)
    g.orient(gpm.ORIENT_CORE)
    assert gpm.motif_count_formula(g, 5) == want
    g.orient(gpm.ORIENT_DEGREE)
    assert gpm.motif_count_formula(g, 5) == want


def big_hub():
    """A vertex joined to all 150 vertices of a sparse random graph: its
    triangles are walked in two tasks of at most 128 of its neighbours."""
    base = graphgen.erdos_renyi(150, 0.05, 11)
    hub = np.full(150, 150, np.int32)
    return graphgen.EdgeList(151, np.concatenate([base.u, hub]),
                             np.concatenate([base.v, np.arange(150, dtype=np.int32)]), "hub150")


def padded(e, n, seed):
    """e with isolated vertices up to n, ids permuted over all n."""
    return graphgen.relabel(graphgen.EdgeList(n, e.u, e.v, f"{e.name}+{n - e.n}"), seed)


@pytest.fixture(scope="module")
def big_hub_counts(gpm):
    e = big_hub()
    off, adj = oracle.canonical_csr(e.n, e.u, e.v)
    return e, [oracle.pattern_count(off, adj, 5, gpm.motif_class_pattern(5, i), True)[0]
               for i in range(21)]


@pytest.mark.parametrize("n", [151, 32768, 40000, 60000, 65536, 65537])
def test_formula_route_hub_and_lds_limit(gpm, big_hub_counts, n):
    """The hub graph alone, and padded with isolated vertices (which change
    no count) to 32,768 vertices (the A^2-row kernel with a bitmap of N(a)
    per wave), 40,000 and 60,000 (one N(a) bitmap shared by the workgroup's
    waves), 65,536, the largest graph whose rows of A^2 fit in LDS (144 KB),
    and 65,537, where the 5-cycle, K_{2,3}, class 16, K5 minus an edge and
    the wheel are counted directly.  All equal the oracle's counts of the
    hub graph."""
    e, want = big_hub_counts
    assert want[18] > 0 and want[19] > 0   # wheels and K5 minus an edge
    print(f"5-motif formula, hub graph on {n} vertices", flush=True)
    g = build(gpm, e if n == e.n else padded(e, n, n))
    assert gpm.motif_count_formula(g, 5) == want
