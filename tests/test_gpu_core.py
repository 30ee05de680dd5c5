"""Core numbers and the core-value orientation (Appendix B.2) on the device
against the oracle's bucket peeling; every count is unchanged by the
orientation."""
import numpy as np
import pytest
import torch

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
    base = graphgen.erdos_renyi(100, 0.06, 3)
    rng = np.random.default_rng(3)
    ends = rng.choice(np.arange(1, 100), size=45, replace=False).astype(np.int32)
    u = np.concatenate([base.u, np.zeros(45, np.int32)])
    v = np.concatenate([base.v, ends])
    return graphgen.EdgeList(100, u, v, "hub")


def graphs():
    return [graphgen.erdos_renyi(300, 0.03, 7),
            hub_graph(),
            graphgen.rmat(12, seed=12),
            graphgen.complete_graph(9),
            graphgen.star_graph(50),
            graphgen.disjoint_union([graphgen.complete_graph(6), graphgen.cycle_graph(9),
                                     graphgen.EdgeList(4, np.zeros(0, np.int32),
                                                       np.zeros(0, np.int32), "isolated")]),
            graphgen.EdgeList(6, np.zeros(0, np.int32), np.zeros(0, np.int32), "empty")]


def core_key(core, deg):
    """(core, degree) packed as the orientation compares them: core above
    S = 31 - bits(largest core) bits, the degree capped below."""
    S = 31 - int(core.max()).bit_length() if core.size else 31
    return (core.astype(np.int64) << S) | np.minimum(deg.astype(np.int64), (1 << S) - 1)


def dag_arcs(g):
    do, da, ds = (t.cpu().numpy() for t in g.dag())
    n = g.n
    src = np.repeat(np.arange(n), np.diff(do))
    assert np.array_equal(src, ds)
    return src.astype(np.int64), da.astype(np.int64)


def dag_arcs_deg(dag, n):
    do, da, _ = (t.cpu().numpy() for t in dag)
    return np.repeat(np.arange(n), np.diff(do)).astype(np.int64), da.astype(np.int64)


@pytest.mark.parametrize("method", ["hindex", "peel"])
@pytest.mark.parametrize("gi", range(7))
def test_core_numbers_and_orientation(gpm, gi, method, monkeypatch):
    """Both core-number methods: the h-index fixed point (the default) and
    the level-synchronous peeling (GPM_CORE_PEEL=1)."""
    if method == "peel":
        monkeypatch.setenv("GPM_CORE_PEEL", "1")
    e = graphs()[gi]
    print(f"graph {gi} {e.name} n={e.n} {method}", flush=True)
    g = build(gpm, e)
    off, adj = oracle.canonical_csr(e.n, e.u, e.v)
    want_core = oracle.core_numbers(off, adj)
    before = [gpm.count(g, gpm.clique(k)) for k in (3, 4, 5)]
    deg_dag = [t.clone() for t in g.dag()]
    deg_maxout = g.max_out_degree
    core = g.orient(gpm.ORIENT_CORE, core_out=True).cpu().numpy()
    assert np.array_equal(core, want_core)
    # every arc goes up in (core, degree, id); each undirected edge once
    a, b = dag_arcs(g)
    assert a.shape[0] == g.m
    key = core_key(core, np.diff(off))
    assert np.all((key[a] < key[b]) | ((key[a] == key[b]) & (a < b)))
    assert set(zip(np.minimum(a, b), np.maximum(a, b))) == \
        set(zip(np.minimum(*dag_arcs_deg(deg_dag, g.n)), np.maximum(*dag_arcs_deg(deg_dag, g.n))))
    assert g.max_out_degree == (int(np.bincount(a, minlength=g.n).max()) if g.m else 0)
    # counts do not depend on the orientation
    assert [gpm.count(g, gpm.clique(k)) for k in (3, 4, 5)] == before
    for k in (3, 4):
        assert gpm.motif_count(g, k) == (oracle.motif3(off, adj) if k == 3 else oracle.motif4(off, adj))
    # back to the degree order: the build's DAG exactly
    assert g.orient(gpm.ORIENT_DEGREE) is None
    for x, y in zip(g.dag(), deg_dag):
        assert torch.equal(x, y)
    assert g.max_out_degree == deg_maxout


def test_core_orientation_all_counts_rmat(gpm):
    """RMAT-14 under the core orientation: cliques up to 6, listings (total
    and checksum), motifs (both routes), diamonds, 4-cycles and a general
    pattern equal the degree order's."""
    e = graphgen.rmat(14, seed=14)
    g = build(gpm, e)
    off, adj = oracle.canonical_csr(e.n, e.u, e.v)

    def snapshot():
        out = [gpm.count(g, gpm.clique(k)) for k in (3, 4, 5, 6)]
        out += [gpm.list_embeddings(g, gpm.clique(k, gpm.VERTEX_INDUCED | gpm.LIST), 1024)[0:3:2]
                for k in (3, 4, 5)]
        out += [gpm.motif_count(g, 3), gpm.motif_count(g, 4), gpm.clique_counts(g, 5)]
        out += [gpm.count(g, gpm.diamond()), gpm.count(g, gpm.cycle4())]
        out += [gpm.motif_count_enum(g, 4),
                gpm.count(g, gpm.pattern(4, [(0, 1), (1, 2), (2, 3)], gpm.VERTEX_INDUCED))]
        return out

    before = snapshot()
    core = g.orient(gpm.ORIENT_CORE, core_out=True).cpu().numpy()
    assert np.array_equal(core, oracle.core_numbers(off, adj))
    assert snapshot() == before
    g.orient(gpm.ORIENT_DEGREE)
    assert snapshot() == before


def test_orient_errors(gpm):
    from paper_2011_03135_amd.binding import GpmError
    g = build(gpm, graphgen.erdos_renyi(50, 0.1, 1))
    with pytest.raises(GpmError) as ei:
        g.orient(7)
    assert ei.value.status == 1


def test_concurrent_orientations_from_two_threads(gpm):
    """Two host threads orient two different graphs on their own streams at
    the same time (the peeling reads its counters through one shared pinned
    buffer); both core arrays equal the oracle's."""
    import threading
    es = [graphgen.rmat(12, seed=12), graphgen.rmat(13, seed=13)]
    gs = [build(gpm, e) for e in es]
    want = []
    for e in es:
        off, adj = oracle.canonical_csr(e.n, e.u, e.v)
        want.append(oracle.core_numbers(off, adj))
    torch.cuda.synchronize()
    got = [None, None]
    errors = []

    def work(i):
        try:
            s = torch.cuda.Stream()
            for _ in range(3):
                with torch.cuda.stream(s):
                    core = gs[i].orient(gpm.ORIENT_CORE, stream=s, core_out=True)
                s.synchronize()
                got[i] = core.cpu().numpy()
                assert np.array_equal(got[i], want[i])
        except Exception as ex:   # reported by the main thread
            errors.append(repr(ex))

    ts = [threading.Thread(target=work, args=(i,)) for i in range(2)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    assert not errors, errors
    for i in range(2):
        assert np.array_equal(got[i], want[i])
