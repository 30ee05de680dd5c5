"""Serving runtime: results in a concurrent mix equal isolated results."""
import pytest

import graphgen
from gpu_util import build

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpm():
    import paper_2011_03135_amd as m
    m.load()
    return m


SCALES = (9, 10, 11, 12)


@pytest.fixture(scope="module")
def edges():
    return [graphgen.rmat(s, seed=1000 + s) for s in SCALES]


@pytest.fixture(scope="module")
def graphs(gpm, edges):
    return [build(gpm, e) for e in edges]


@pytest.fixture(scope="module")
def oracle_counts(edges):
    """The oracle's answer to every query on every graph."""
    import oracle
    out = {}
    for gi, e in enumerate(edges):
        off, adj = oracle.canonical_csr(e.n, e.u, e.v)
        out[(gi, "TC")] = [oracle.clique_count(off, adj, 3)]
        out[(gi, "4-clique")] = [oracle.clique_count(off, adj, 4)]
        out[(gi, "3-motif")] = oracle.motif3(off, adj)
        out[(gi, "4-motif")] = oracle.motif4(off, adj)
    return out


def isolated(gpm, g, name):
    if name == "TC":
        return [gpm.count(g, gpm.clique(3))]
    if name == "4-clique":
        return [gpm.count(g, gpm.clique(4))]
    return gpm.motif_count(g, 3 if name == "3-motif" else 4)


def test_mix_equals_isolated_and_oracle(gpm, graphs, oracle_counts):
    """Every served result equals the oracle's count and the same query run
    alone on the device."""
    from paper_2011_03135_amd.serve import QUERIES, run_load
    want = {}
    for gi in range(len(graphs)):
        for qi, q in enumerate(QUERIES):
            want[(gi, qi)] = oracle_counts[(gi, q[0])]
            assert isolated(gpm, graphs[gi], q[0]) == want[(gi, qi)], (gi, q[0])
    stats, per = run_load(graphs, rate=2000.0, n_requests=400, n_warmup=40, seed=5,
                          max_slots=4, pool_bytes=1 << 30)
    assert stats["failed"] == 0
    for gi, qi, r in per:
        assert r.status == 0
        got = r.counts()
        assert got == want[(gi, qi)], (gi, qi, got)
        assert r.t_submit <= r.t_admit <= r.t_done
        assert 0.0 <= r.d_start <= r.d_end


def test_requests_overlap_on_device(gpm, graphs, oracle_counts):
    """Requests queued together run side by side: with four slots, some two
    requests' device spans (events recorded on their streams before and after
    their work) overlap, and so do their host admission-to-completion
    intervals; every result still equals the oracle's."""
    from paper_2011_03135_amd.binding import QUERY_MOTIF, Server
    srv = Server(max_slots=4, pool_bytes=1 << 30)
    gi = len(graphs) - 1
    ids = [srv.submit(graphs[gi], QUERY_MOTIF, 4, tag=i) for i in range(16)]
    got = {}
    while len(got) < len(ids):
        for r in srv.poll():
            got[r.tag] = r
    srv.close()
    for r in got.values():
        assert r.status == 0
        assert r.counts() == oracle_counts[(gi, "4-motif")]

    def overlapping(spans):
        spans = sorted(spans)
        return sum(1 for (a0, b0), (a1, b1) in zip(spans, spans[1:]) if a1 < b0)

    dev = overlapping([(r.d_start, r.d_end) for r in got.values()])
    host = overlapping([(r.t_admit, r.t_done) for r in got.values()])
    print(f"overlapping neighbours: device {dev}, host {host}", flush=True)
    assert dev >= 1
    assert host >= 1


def test_small_pool_defers(gpm, graphs):
    """A pool that holds one request at a time still serves every request."""
    from paper_2011_03135_amd.binding import QUERY_CLIQUE, Server
    g = graphs[-1]
    ws = gpm.workspace_bytes(g, gpm.clique(4))
    srv = Server(max_slots=4, pool_bytes=ws + 4 * 256 + 4096)   # room for one workspace
    ids = [srv.submit(g, QUERY_CLIQUE, 4, tag=i) for i in range(12)]
    got = {}
    while len(got) < len(ids):
        for r in srv.poll():
            got[r.tag] = r
    srv.close()
    want = [gpm.count(g, gpm.clique(4))]
    for i in range(12):
        assert got[i].status == 0
        assert got[i].counts() == want
    # admissions never overlapped: each started after the previous finished
    spans = sorted((r.t_admit, r.t_done) for r in got.values())
    for (a0, d0), (a1, d1) in zip(spans, spans[1:]):
        assert a1 >= d0 - 1e-4


def test_rejects_oversized_and_invalid(gpm, graphs):
    from paper_2011_03135_amd.binding import QUERY_CLIQUE, QUERY_MOTIF, Server
    srv = Server(max_slots=2, pool_bytes=1 << 16)
    with pytest.raises(gpm.GpmError):
        srv.submit(graphs[-1], QUERY_MOTIF, 4)      # workspace larger than the pool
    with pytest.raises(gpm.GpmError):
        srv.submit(graphs[0], QUERY_CLIQUE, 10)     # unsupported clique size
    srv.close()
