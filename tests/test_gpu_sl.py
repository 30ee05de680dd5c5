"""Edge-induced diamond and 4-cycle counting and listing against the oracle."""
import json
import os

import numpy as np
import pytest

import graphgen
import oracle
from oracle import canonical_csr
from gpu_util import build

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "rmat_counts.json")


@pytest.fixture(scope="module")
def gpm():
    import paper_2011_03135_amd as m
    m.load()
    return m


def edge_sets(name, rows):
    out = set()
    for r in rows:
        a, b, c, d = (int(x) for x in r)
        if name == "diamond":
            F = [(a, b), (a, c), (a, d), (b, c), (b, d)]
        else:
            F = [(a, b), (b, c), (c, d), (d, a)]
        out.add(frozenset(tuple(sorted(e)) for e in F))
    return out


def cases():
    return [
        graphgen.complete_graph(8),
        graphgen.complete_bipartite(6, 9),
        graphgen.erdos_renyi(150, 0.08, 41),
        graphgen.rmat(11, seed=43),
        graphgen.complete_bipartite(40, 300),     # heavy apexes, many 4-cycles
        graphgen.cycle_graph(4),
        graphgen.star_graph(50),
    ]


PATS = ("diamond", "4-cycle")


@pytest.mark.parametrize("case", range(7))
@pytest.mark.parametrize("name", PATS)
def test_sl_count_and_list(gpm, case, name):
    e = cases()[case]
    print(f"sl {name} case {case} {e.name}", flush=True)
    g = build(gpm, e)
    off, adj = canonical_csr(e.n, e.u, e.v)
    ofn = oracle.list_diamonds if name == "diamond" else oracle.list_c4
    total, chk, rows = ofn(off, adj, cap=2 * 10 ** 6)
    pat = gpm.diamond() if name == "diamond" else gpm.cycle4()
    assert gpm.count(g, pat) == total
    lpat = gpm.diamond(gpm.EDGE_INDUCED | gpm.LIST) if name == "diamond" else \
        gpm.cycle4(gpm.EDGE_INDUCED | gpm.LIST)
    t, w, c, got = gpm.list_embeddings(g, lpat, 2 * 10 ** 6)
    assert (t, c) == (total, chk)
    if total <= 2 * 10 ** 6:
        assert w == total
        assert edge_sets(name, got.cpu().tolist()) == edge_sets(name, rows.tolist())


@pytest.mark.parametrize("name", PATS)
def test_sl_truncated(gpm, name):
    e = graphgen.erdos_renyi(120, 0.15, 9)
    g = build(gpm, e)
    off, adj = canonical_csr(e.n, e.u, e.v)
    ofn = oracle.list_diamonds if name == "diamond" else oracle.list_c4
    total, chk, rows = ofn(off, adj, cap=10 ** 6)
    valid = edge_sets(name, rows.tolist())
    lpat = gpm.diamond(gpm.EDGE_INDUCED | gpm.LIST) if name == "diamond" else \
        gpm.cycle4(gpm.EDGE_INDUCED | gpm.LIST)
    cap = total // 5
    t, w, c, got = gpm.list_embeddings(g, lpat, cap)
    assert (t, w, c) == (total, cap, chk)
    sets = edge_sets(name, got.cpu().tolist())
    assert len(sets) == cap and sets <= valid


def test_rmat18_sl_golden(gpm):
    if not os.path.exists(GOLDEN):
        pytest.skip("golden counts not generated")
    with open(GOLDEN) as f:
        gold = json.load(f).get("rmat18", {})
    if "sl_4-cycle" not in gold:
        pytest.skip("rmat18 listing golden values not generated")
    g = build(gpm, graphgen.rmat(18, seed=18))
    for name, pat, lpat in (("diamond", gpm.diamond(), gpm.diamond(gpm.EDGE_INDUCED | gpm.LIST)),
                            ("4-cycle", gpm.cycle4(), gpm.cycle4(gpm.EDGE_INDUCED | gpm.LIST))):
        want = gold[f"sl_{name}"]
        assert gpm.count(g, pat) == want["total"]
        t, w, c, _ = gpm.list_embeddings(g, lpat, 1 << 20)
        assert (t, w, c) == (want["total"], min(1 << 20, want["total"]), want["checksum"])
