"""Plain-path tuning (gpm_tuning): counts never depend on it, its ranges are
checked, workspace sizes follow it, and the autotuner returns a valid
setting that it leaves in the handle."""
import ctypes
from math import comb

import pytest
import torch

import graphgen
import oracle
from gpu_util import build

pytestmark = pytest.mark.gpu

DEFAULT = {"tc_tau": [8192, 16384, 65536], "tc_blocks_per_cu": [32, 8, 4],
           "clique_wave_blocks_per_cu": 32, "lg5_slice": 1 << 20}
FINE = {"tc_tau": [2048] * 3, "tc_blocks_per_cu": [1] * 3, "clique_wave_blocks_per_cu": 8,
        "lg5_slice": 1 << 14}
COARSE = {"tc_tau": [1 << 24] * 3, "tc_blocks_per_cu": [64] * 3,
          "clique_wave_blocks_per_cu": 1024, "lg5_slice": 1 << 28}


@pytest.fixture(scope="module")
def gpm():
    import paper_2011_03135_amd as m
    m.load()
    return m


def snapshot(gpm, g):
    """Every count whose schedule the tuning changes: triangles (count,
    listing total and checksum, per-edge counts through the 4-motifs), 4-
    and 5-cliques alone and fused."""
    out = [gpm.count(g, gpm.clique(k)) for k in (3, 4, 5)]
    total, _, checksum, _ = gpm.list_embeddings(
        g, gpm.clique(3, gpm.VERTEX_INDUCED | gpm.LIST), 1024)
    out += [total, checksum, gpm.clique_counts(g, 5), gpm.motif_count(g, 4)]
    return out


def test_default_tuning(gpm):
    g = build(gpm, graphgen.erdos_renyi(200, 0.05, 1))
    assert g.tuning() == DEFAULT


@pytest.mark.parametrize("case", ["er", "rmat12", "k300"])
def test_counts_do_not_depend_on_tuning(gpm, case):
    e = {"er": lambda: graphgen.erdos_renyi(4096, 0.004, 1),
         "rmat12": lambda: graphgen.rmat(12, seed=12),
         "k300": lambda: graphgen.complete_graph(300)}[case]()
    print(f"tuning invariance on {e.name}", flush=True)
    g = build(gpm, e)
    want = snapshot(gpm, g)
    if case == "k300":
        assert want[:3] == [comb(300, 3), comb(300, 4), comb(300, 5)]
    if case == "er":
        off, adj = oracle.canonical_csr(e.n, e.u, e.v)
        assert want[0] == oracle.clique_count(off, adj, 3)
    for t in (FINE, COARSE):
        g.set_tuning(**t)
        assert g.tuning() == t
        assert snapshot(gpm, g) == want
    g.set_tuning(**DEFAULT)
    assert snapshot(gpm, g) == want


def test_tuning_ranges(gpm):
    from paper_2011_03135_amd.binding import GpmError
    g = build(gpm, graphgen.erdos_renyi(100, 0.1, 2))
    bad = [{"tc_tau": [2047, 16384, 65536]}, {"tc_tau": [8192, 16384, (1 << 24) + 1]},
           {"tc_blocks_per_cu": [0, 8, 4]}, {"tc_blocks_per_cu": [32, 65, 4]},
           {"clique_wave_blocks_per_cu": 7}, {"clique_wave_blocks_per_cu": 1025},
           {"lg5_slice": (1 << 14) - 1}, {"lg5_slice": (1 << 28) + 1}]
    for kw in bad:
        with pytest.raises(GpmError) as ei:
            g.set_tuning(**kw)
        assert ei.value.status == 1
        assert g.tuning() == DEFAULT


def test_workspace_follows_tuning(gpm):
    """A workspace sized under the default chunks is too small once the
    chunks shrink: the call refuses it (GPM_OUT_OF_MEMORY) and writes
    nothing."""
    lib = gpm.load()
    g = build(gpm, graphgen.rmat(12, seed=12))
    p = gpm.clique(3)
    small = gpm.workspace_bytes(g, p)
    ws = torch.empty(small, dtype=torch.uint8, device="cuda")
    g.set_tuning(tc_tau=[2048] * 3)
    assert gpm.workspace_bytes(g, p) > small
    out = torch.full((1,), -7, dtype=torch.int64, device="cuda")
    rc = lib.gpm_count(g.handle, ctypes.byref(p), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                       ctypes.c_void_p(out.data_ptr()), None)
    assert rc == 2
    assert int(out.item()) == -7


@pytest.mark.parametrize("scale", [12, 14])
def test_autotune(gpm, scale):
    g = build(gpm, graphgen.rmat(scale, seed=scale))
    want = snapshot(gpm, g)
    print(f"autotune rmat{scale}", flush=True)
    t = g.autotune()
    assert g.tuning() == t
    assert all(2048 <= x <= 1 << 24 for x in t["tc_tau"])
    assert all(1 <= x <= 64 for x in t["tc_blocks_per_cu"])
    assert 8 <= t["clique_wave_blocks_per_cu"] <= 1024
    assert (1 << 14) <= t["lg5_slice"] <= 1 << 28
    assert snapshot(gpm, g) == want


def test_autotune_slices_on_a_graph_with_large_roots(gpm):
    """K_300 has roots of out-degree above 256, so the 5-clique slices are
    tuned too; the counts stay C(300, k)."""
    g = build(gpm, graphgen.complete_graph(300))
    t = g.autotune()
    assert g.tuning() == t
    assert [gpm.count(g, gpm.clique(k)) for k in (3, 4, 5)] == \
        [comb(300, 3), comb(300, 4), comb(300, 5)]


@pytest.mark.parametrize("case", ["edgeless", "one_edge", "star"])
def test_autotune_degenerate_graphs(gpm, case):
    """Graphs with no triangle work at all: the tuner still returns a valid
    setting and the counts stay exact."""
    import numpy as np
    e = {"edgeless": lambda: graphgen.EdgeList(5, np.zeros(0, np.int32), np.zeros(0, np.int32),
                                               "edgeless"),
         "one_edge": lambda: graphgen.EdgeList(2, np.array([0], np.int32),
                                               np.array([1], np.int32), "one_edge"),
         "star": lambda: graphgen.star_graph(40)}[case]()
    g = build(gpm, e)
    t = g.autotune()
    assert g.tuning() == t
    assert [gpm.count(g, gpm.clique(k)) for k in (3, 4, 5)] == [0, 0, 0]
