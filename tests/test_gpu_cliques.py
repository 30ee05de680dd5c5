"""Device graph build and clique counting/listing against the CPU oracle."""
import json
import os

import math

import numpy as np
import pytest
import torch

import graphgen
import oracle
from oracle import canonical_csr
from gpu_util import build, degree_rank_dag

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "rmat_counts.json")


@pytest.fixture(scope="module")
def gpm():
    import paper_2011_03135_amd as m
    m.load()
    return m


def noisy_stream(n, pairs, seed):
    """A raw stream holding every pair in both directions, repeats and loops."""
    rng = np.random.default_rng(seed)
    a = np.array([p[0] for p in pairs], np.int64)
    b = np.array([p[1] for p in pairs], np.int64)
    rep = rng.integers(1, 4, size=a.shape[0])
    a2, b2 = np.repeat(a, rep), np.repeat(b, rep)
    flip = rng.integers(0, 2, size=a2.shape[0]).astype(bool)
    u = np.where(flip, b2, a2)
    v = np.where(flip, a2, b2)
    loops = rng.integers(0, n, size=max(1, n // 10))
    u = np.concatenate([u, loops])
    v = np.concatenate([v, loops])
    perm = rng.permutation(u.shape[0])
    return graphgen.EdgeList(n, u[perm].astype(np.int32), v[perm].astype(np.int32), "noisy")


def build_cases():
    star = graphgen.star_graph(5000)                      # one 5000-entry row: bitmap sorter
    star_pairs = list(zip(star.u.tolist(), star.v.tolist()))
    mid = graphgen.star_graph(700)                        # a 700-entry row: LDS sorter
    return [
        graphgen.erdos_renyi(300, 0.05, 3),
        graphgen.rmat(12, seed=7),
        noisy_stream(5001, star_pairs, 1),
        noisy_stream(701, list(zip(mid.u.tolist(), mid.v.tolist())), 2),
        graphgen.complete_graph(40),
        graphgen.EdgeList(5, np.zeros(0, np.int32), np.zeros(0, np.int32), "empty"),
        wide_id_range(),
    ]


def wide_id_range():
    """n = 1.3M ids (above the on-chip bitmap of the long-row sorter): a
    3000-entry row plus random edges, each listed twice."""
    n = 1_300_000
    rng = np.random.default_rng(11)
    hub = np.zeros(3000, np.int64)
    ends = rng.choice(np.arange(1, n), size=3000, replace=False)
    a = rng.integers(0, n, size=20000)
    b = rng.integers(0, n, size=20000)
    u = np.concatenate([hub, ends, a, b]).astype(np.int32)
    v = np.concatenate([ends, hub, b, a]).astype(np.int32)
    return graphgen.EdgeList(n, u, v, "wide")


@pytest.mark.parametrize("case", range(7))
def test_build_matches_oracle(gpm, case):
    e = build_cases()[case]
    print(f"build case {case} {e.name} n={e.n} E={e.num_input_edges}", flush=True)
    g = build(gpm, e)
    off_ref, adj_ref = canonical_csr(e.n, e.u, e.v)
    off, adj = (t.cpu().numpy() for t in g.csr())
    assert g.n == e.n and g.m == adj_ref.shape[0] // 2
    assert np.array_equal(off, off_ref.astype(np.int32))
    assert np.array_equal(adj, adj_ref)
    dag_off, dag_adj, dag_src = (t.cpu().numpy() for t in g.dag())
    src, dst = degree_rank_dag(off_ref, adj_ref)
    assert np.array_equal(dag_adj, dst.astype(np.int32))
    assert np.array_equal(dag_src, src.astype(np.int32))
    assert np.array_equal(np.diff(dag_off), np.bincount(src, minlength=e.n))
    assert g.max_degree == (int(np.diff(off_ref).max()) if e.n else 0)
    assert g.max_out_degree == int(np.diff(dag_off).max())


@pytest.mark.parametrize("case", range(4))
def test_from_csr_equals_build(gpm, case):
    """A graph made from a canonical CSR equals the one built from the edge
    stream: same CSR, DAG and counts."""
    e = [graphgen.rmat(12, seed=5), graphgen.erdos_renyi(500, 0.05, 3),
         graphgen.complete_graph(40), graphgen.star_graph(50)][case]
    g = build(gpm, e)
    off, adj = g.csr()
    h = gpm.Graph.from_csr(e.n, off.clone(), adj.clone(), validate=True)
    assert (h.n, h.m, h.max_degree, h.max_out_degree) == (g.n, g.m, g.max_degree,
                                                            g.max_out_degree)
    for a, b in zip(g.dag(), h.dag()):
        assert torch.equal(a, b)
    for k in (3, 4, 5):
        assert gpm.count(h, gpm.clique(k)) == gpm.count(g, gpm.clique(k))
    assert gpm.motif_count(h, 4) == gpm.motif_count(g, 4)


def test_from_csr_rejects_non_canonical(gpm):
    e = graphgen.erdos_renyi(200, 0.05, 4)
    g = build(gpm, e)
    off, adj = (t.clone() for t in g.csr())
    bad_cases = []
    a = adj.clone()
    a[0], a[1] = adj[1], adj[0]                     # row 0 out of order
    bad_cases.append((off, a, True))
    a = adj.clone()
    a[5] = 10 ** 6                                  # id out of range
    bad_cases.append((off, a, False))
    o = off.clone()
    o[-1] = o[-1] - 2                               # offsets inconsistent with nnz
    bad_cases.append((o, adj, False))
    # one direction of an edge missing: move the last arc of a row to the
    # next id, which is not yet a neighbour (rows stay sorted, nnz even)
    oh, ah = off.cpu().numpy(), adj.cpu().numpy()
    r = next(r for r in range(e.n) if oh[r + 1] > oh[r]
             and ah[oh[r + 1] - 1] + 1 < e.n and ah[oh[r + 1] - 1] + 1 != r)
    a = adj.clone()
    last = int(oh[r + 1]) - 1
    a[last] = a[last] + 1
    bad_cases.append((off, a, True))
    for o_, a_, validate in bad_cases:
        with pytest.raises(gpm.GpmError) as ei:
            gpm.Graph.from_csr(e.n, o_, a_, validate=validate)
        assert ei.value.status == 6
    with pytest.raises(gpm.GpmError) as ei:          # odd nnz
        gpm.Graph.from_csr(e.n, off, adj[:-1].clone())
    assert ei.value.status == 5


def test_build_rejects_out_of_range(gpm):
    e = graphgen.EdgeList(4, np.array([0, 1], np.int32), np.array([1, 4], np.int32))
    with pytest.raises(gpm.GpmError) as ei:
        build(gpm, e)
    assert ei.value.status == 6


def clique_cases():
    return [
        graphgen.complete_graph(12),
        graphgen.complete_graph(70),                        # out-degree 69: workgroup class
        graphgen.complete_multipartite([3, 5, 2, 7, 4, 6]),
        graphgen.erdos_renyi(200, 0.15, 11),
        graphgen.rmat(12, seed=5),
        graphgen.rmat(14, seed=14),
        graphgen.star_graph(100),
        graphgen.EdgeList(5, np.zeros(0, np.int32), np.zeros(0, np.int32), "empty"),
    ]


@pytest.mark.parametrize("case", range(8))
def test_clique_counts(gpm, case):
    e = clique_cases()[case]
    g = build(gpm, e)
    off, adj = canonical_csr(e.n, e.u, e.v)
    # 7- and 8-cliques where the oracle finishes quickly (not the RMAT cases)
    ks = (3, 4, 5, 6) if e.name.startswith("rmat") else (3, 4, 5, 6, 7, 8)
    complete = e.name[1:].isdigit()     # K_n: the closed form C(n, k)
    for k in ks:
        print(f"clique case {case} {e.name} k={k}", flush=True)
        want = math.comb(e.n, k) if complete else oracle.clique_count(off, adj, k)
        assert gpm.count(g, gpm.clique(k)) == want, (e.name, k)


@pytest.mark.parametrize("n", [40, 66, 100])
def test_dense_local_graphs_large_k(gpm, n):
    """k = 6..9 on complete graphs (local rows of 1 or 2 words, level-1 sets
    of up to n - 2 members)."""
    g = build(gpm, graphgen.complete_graph(n))
    for k in (6, 7, 8, 9) if n <= 66 else (6, 7, 8):
        print(f"complete graph n={n} k={k}", flush=True)
        assert gpm.count(g, gpm.clique(k)) == math.comb(n, k)


def test_large_k_multipartite(gpm):
    """Complete multipartite graph with out-degrees above 256 (5- to 8-word
    local rows): 6-cliques = e_6(part sizes)."""
    parts = [40, 35, 30, 25, 20, 45, 50, 15, 10, 60]
    g = build(gpm, graphgen.complete_multipartite(parts))
    print(f"multipartite max_out={g.max_out_degree}", flush=True)
    assert gpm.count(g, gpm.clique(6)) == elementary_symmetric(parts, 6)


@pytest.mark.parametrize("n", [130, 200, 257, 300, 520, 700])
def test_dense_local_graphs(gpm, n):
    """Complete graphs put every root's local graph at full density; the
    roots' out-degrees cover local rows of 3 to 11 words."""
    g = build(gpm, graphgen.complete_graph(n))
    for k in (4, 5):
        print(f"complete graph n={n} k={k}", flush=True)
        assert gpm.count(g, gpm.clique(k)) == math.comb(n, k)


def elementary_symmetric(parts, k):
    e = [1] + [0] * k
    for x in parts:
        for j in range(k, 0, -1):
            e[j] += e[j - 1] * x
    return e[k]


@pytest.mark.parametrize("parts", [[20] * 20, [7, 13, 25, 40, 3, 60, 90, 30, 50, 22, 18, 35, 11, 70]])
def test_dense_multipartite_local_graphs(gpm, parts):
    """Complete multipartite graphs: k-cliques = e_k(part sizes); local graphs
    are dense but not complete, with out-degrees up to about 470."""
    g = build(gpm, graphgen.complete_multipartite(parts))
    for k in (3, 4, 5):
        print(f"multipartite {len(parts)} parts k={k} max_out={g.max_out_degree}", flush=True)
        assert gpm.count(g, gpm.clique(k)) == elementary_symmetric(parts, k)


@pytest.mark.parametrize("case", range(8))
def test_fused_clique_counts(gpm, case):
    """One local-graph pass gives the same triangle, 4- and 5-clique counts
    as the per-size calls and the oracle."""
    e = clique_cases()[case]
    g = build(gpm, e)
    off, adj = canonical_csr(e.n, e.u, e.v)
    want = [oracle.clique_count(off, adj, k) for k in (3, 4, 5)]
    print(f"fused case {case} {e.name}", flush=True)
    assert gpm.clique_counts(g, 5) == want
    assert gpm.clique_counts(g, 4) == want[:2]


@pytest.mark.parametrize("n", [70, 300, 700])
def test_fused_clique_counts_dense(gpm, n):
    g = build(gpm, graphgen.complete_graph(n))
    assert gpm.clique_counts(g, 5) == [math.comb(n, k) for k in (3, 4, 5)]


def test_fused_clique_counts_rmat_golden(gpm):
    gold = _golden().get("rmat18")
    if not gold or "clique5" not in gold:
        pytest.skip("golden counts for rmat18 not generated")
    g = build(gpm, graphgen.rmat(18, seed=18))
    assert gpm.clique_counts(g, 5) == [gold["clique3"], gold["clique4"], gold["clique5"]]


def test_er_workload_triangles(gpm):
    """Erdos-Renyi G(4096, 0.004), seed 1."""
    e = graphgen.erdos_renyi(4096, 0.004, 1)
    g = build(gpm, e)
    off, adj = canonical_csr(e.n, e.u, e.v)
    assert gpm.count(g, gpm.clique(3)) == oracle.triangle_count(off, adj)


def test_generic_path_high_out_degree(gpm):
    """Out-degrees above 1024 take the depth-first kernel."""
    e = graphgen.complete_multipartite([2] * 520)
    g = build(gpm, e)
    assert g.max_out_degree > 1024
    off, adj = canonical_csr(e.n, e.u, e.v)
    assert gpm.count(g, gpm.clique(3)) == oracle.clique_count(off, adj, 3)


def test_relabel_invariance(gpm):
    e = graphgen.rmat(13, seed=3)
    a = build(gpm, e)
    b = build(gpm, graphgen.relabel(e, 77))
    for k in (3, 4, 5):
        assert gpm.count(a, gpm.clique(k)) == gpm.count(b, gpm.clique(k))


@pytest.mark.parametrize("k", [3, 4, 5])
def test_clique_listing(gpm, k):
    e = graphgen.erdos_renyi(60, 0.35, 4)
    g = build(gpm, e)
    off, adj = canonical_csr(e.n, e.u, e.v)
    total, chk, rows = oracle.clique_list(off, adj, k, cap=10 ** 6)
    t, w, c, got = gpm.list_embeddings(g, gpm.clique(k, gpm.VERTEX_INDUCED | gpm.LIST), 10 ** 6)
    assert (t, w, c) == (total, total, chk)
    assert {tuple(sorted(r)) for r in got.cpu().tolist()} == {tuple(sorted(r)) for r in rows.tolist()}
    # truncated: totals and checksum still exact, every written row a clique
    cap = max(1, total // 3)
    t, w, c, got = gpm.list_embeddings(g, gpm.clique(k, gpm.VERTEX_INDUCED | gpm.LIST), cap)
    assert (t, w, c) == (total, min(cap, total), chk)
    A = set(map(tuple, np.stack([np.repeat(np.arange(e.n), np.diff(off)), adj], 1).tolist()))
    for r in got.cpu().tolist():
        assert len(set(r)) == k
        assert all((a, b) in A for i, a in enumerate(r) for b in r[i + 1:])


@pytest.mark.parametrize("k", [3, 4])
def test_edge_induced_clique_listing_key(gpm, k):
    """A clique's vertex- and edge-induced embeddings are the same vertex
    sets, and the listing keys both by the ascending vertex tuple: the
    edge-induced flag gives the oracle's clique listing too."""
    e = graphgen.erdos_renyi(60, 0.35, 4)
    g = build(gpm, e)
    off, adj = canonical_csr(e.n, e.u, e.v)
    total, chk, rows = oracle.clique_list(off, adj, k, cap=10 ** 6)
    t, w, c, got = gpm.list_embeddings(g, gpm.clique(k, gpm.EDGE_INDUCED | gpm.LIST), 10 ** 6)
    assert (t, w, c) == (total, total, chk)
    assert {tuple(sorted(r)) for r in got.cpu().tolist()} == {tuple(sorted(r)) for r in rows.tolist()}


def hub_graph(seed=3):
    """Roots in every out-degree class: 300 hubs (350 leaf edges each, random
    hub-hub edges p = 0.15), root A adjacent to all hubs (out-degree 300,
    above 256), root B to 150 of them (out-degree 150), 3000 leaves."""
    rng = np.random.default_rng(seed)
    H, L = 300, 3000
    hubs = np.arange(H)
    a_root, b_root = H, H + 1
    leaf0 = H + 2
    us, vs = [], []
    for h in hubs:
        lv = leaf0 + rng.choice(L, 350, replace=False)
        us.append(np.full(350, h)); vs.append(lv)
    iu, ju = np.triu_indices(H, 1)
    keep = rng.random(iu.shape[0]) < 0.15
    us.append(iu[keep]); vs.append(ju[keep])
    us.append(np.full(H, a_root)); vs.append(hubs)
    bsel = rng.choice(H, 150, replace=False)
    us.append(np.full(150, b_root)); vs.append(bsel)
    u = np.concatenate(us).astype(np.int32)
    v = np.concatenate(vs).astype(np.int32)
    return graphgen.EdgeList(leaf0 + L, u, v, "hubs")


@pytest.mark.parametrize("gname", ["rmat14", "hubs"])
@pytest.mark.parametrize("k", [3, 4, 5])
def test_clique_listing_classes(gpm, k, gname):
    """Listing through every out-degree class (<= 64, 65..256, 257..1024):
    exact total and checksum, truncated rows that are cliques."""
    e = graphgen.rmat(14, seed=14) if gname == "rmat14" else hub_graph()
    g = build(gpm, e)
    off, adj = canonical_csr(e.n, e.u, e.v)
    print(f"{gname} k={k} max_out={g.max_out_degree}", flush=True)
    if gname == "hubs":
        assert g.max_out_degree > 256
    total, chk, _ = oracle.clique_list(off, adj, k, cap=0)
    cap = 1 << 16
    t, w, c, got = gpm.list_embeddings(g, gpm.clique(k, gpm.VERTEX_INDUCED | gpm.LIST), cap)
    assert (t, w, c) == (total, min(cap, total), chk)
    rows = got.cpu().numpy().astype(np.int64)
    assert rows.shape == (min(cap, total), k)
    assert (np.sort(rows, axis=1)[:, 1:] > np.sort(rows, axis=1)[:, :-1]).all()
    A = set((np.repeat(np.arange(e.n), np.diff(off)) * e.n + adj).tolist())
    for i in range(k):
        for j in range(i + 1, k):
            assert all(int(x) in A for x in rows[:, i] * e.n + rows[:, j])


def _golden():
    if not os.path.exists(GOLDEN):
        pytest.skip("golden counts not generated")
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.mark.parametrize("scale", [18, 20])
def test_rmat_clique_counts_golden(gpm, scale):
    gold = _golden().get(f"rmat{scale}")
    if gold is None or "clique5" not in gold:
        pytest.skip("golden counts for this scale not generated")
    e = graphgen.rmat(scale, seed=scale)
    g = build(gpm, e)
    assert g.m == gold["m"]
    for k in (3, 4, 5):
        print(f"rmat{scale} k={k}", flush=True)
        assert gpm.count(g, gpm.clique(k)) == gold[f"clique{k}"], k


@pytest.mark.parametrize("case", [1, 3, 4])
def test_without_local_graphs(gpm, case, monkeypatch):
    """GPM_LG=0 sends k >= 4 to the depth-first search without local graphs:
    the same counts, and the same listing totals and checksums."""
    e = clique_cases()[case]
    print(f"clique case {case} {e.name}", flush=True)
    g = build(gpm, e)
    want = {k: gpm.count(g, gpm.clique(k)) for k in (4, 5)}
    lists = {k: gpm.list_embeddings(g, gpm.clique(k, gpm.VERTEX_INDUCED | gpm.LIST), 1 << 16)[:3]
             for k in (4, 5)}
    want3 = gpm.count(g, gpm.clique(3))
    monkeypatch.setenv("GPM_LG", "0")
    for k in (4, 5):
        assert gpm.count(g, gpm.clique(k)) == want[k], k
        got = gpm.list_embeddings(g, gpm.clique(k, gpm.VERTEX_INDUCED | gpm.LIST), 1 << 16)
        assert got[0] == lists[k][0] and got[2] == lists[k][2], k
    assert gpm.clique_counts(g, 4) == [want3, want[4]]
    assert gpm.clique_counts(g, 5) == [want3, want[4], want[5]]


def test_nine_cliques(gpm, monkeypatch):
    """9-cliques: the oracle on a dense random graph (wave class, and the
    depth-first kernel without local graphs), e_9 of the part sizes on a
    complete multipartite graph, and the 9-clique listing's total and
    checksum."""
    e = graphgen.erdos_renyi(120, 0.55, 19)
    g = build(gpm, e)
    off, adj = canonical_csr(e.n, e.u, e.v)
    want = oracle.clique_count(off, adj, 9)
    print(f"ER 9-cliques {want}", flush=True)
    assert want > 0
    assert gpm.count(g, gpm.clique(9)) == want
    total, chk, _ = oracle.clique_list(off, adj, 9, cap=16)
    t, w, c, _ = gpm.list_embeddings(g, gpm.clique(9, gpm.VERTEX_INDUCED | gpm.LIST), 16)
    assert (t, w, c) == (total, min(16, total), chk)
    parts = [5] * 12 + [3] * 4
    gm = build(gpm, graphgen.complete_multipartite(parts))
    assert gpm.count(gm, gpm.clique(9)) == elementary_symmetric(parts, 9)
    monkeypatch.setenv("GPM_LG", "0")
    assert gpm.count(g, gpm.clique(9)) == want
