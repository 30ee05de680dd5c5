"""The allocation-free batch entry point (gpm_batch_motif_count_static,
for callers that cannot allocate): called through the C ABI, it gives the
same per-graph motif counts as gpm_batch_motif_count with a caller
workspace, on two calls in a row (the second on a smaller batch, so the
static scratch holds the first call's leftovers), and it rejects a batch
larger than its scratch before enqueuing anything."""
import ctypes

import numpy as np
import pytest
import torch

import graphgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpm():
    import paper_2011_03135_amd as m
    m.load()
    return m


def batch_graph(gpm, G, seed):
    b = graphgen.rgg_batch(G, seed=seed)
    g = gpm.Graph.build(b.n, torch.from_numpy(b.u).cuda(), torch.from_numpy(b.v).cuda())
    voff = torch.from_numpy(b.voff.astype(np.int32)).cuda()
    return g, voff


def call_static(gpm, g, voff, k, out):
    lib = gpm.binding.load()
    G = voff.shape[0] - 1
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return lib.gpm_batch_motif_count_static(g.handle, ctypes.c_void_p(voff.data_ptr()), G, k,
                                            ctypes.c_void_p(out.data_ptr()), s)


@pytest.mark.parametrize("k", [4, 3])
def test_static_equals_workspace_entry(gpm, k):
    width = 7 if k == 4 else 3
    for G, seed in ((3000, 2020), (700, 7)):       # second call: a smaller batch
        print(f"static batch k={k} G={G} seed={seed}", flush=True)
        g, voff = batch_graph(gpm, G, seed)
        want = gpm.batch_motif_count(g, voff, k)
        got = torch.full((G, width), -1, dtype=torch.int64, device="cuda")
        assert call_static(gpm, g, voff, k, got) == 0
        torch.cuda.synchronize()
        assert torch.equal(got, want)
        assert bool((got[:, -1] == 0).all())


def test_static_rejects_oversized_batch(gpm):
    g, voff = batch_graph(gpm, 50, 3)
    big = gpm.binding.BATCH_STATIC_MAX_GRAPHS + 1
    # a voff tensor of the oversized length; the call must fail on the host
    voff_big = torch.zeros(big + 1, dtype=torch.int32, device="cuda")
    out = torch.full((big, 7), -1, dtype=torch.int64, device="cuda")
    assert call_static(gpm, g, voff_big, 4, out) == 2      # GPM_OUT_OF_MEMORY
    torch.cuda.synchronize()
    assert bool((out == -1).all())
    err = gpm.binding.load().gpm_last_error().decode()
    assert "static scratch" in err
