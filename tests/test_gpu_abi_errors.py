"""Error paths of the C ABI that need a device graph: a workspace smaller
than the size query returns GPM_OUT_OF_MEMORY before anything is enqueued,
so the caller's output buffers keep their contents."""
import ctypes

import pytest
import torch

import graphgen
from gpu_util import build

pytestmark = pytest.mark.gpu

OOM = 2
SENTINEL = 0x5A5A5A5A5A5A5A5A


@pytest.fixture(scope="module")
def gpm():
    import paper_2011_03135_amd as m
    m.load()
    return m


@pytest.fixture(scope="module")
def graph(gpm):
    return build(gpm, graphgen.rmat(10, seed=77))


def small_ws(need):
    """A workspace 256 bytes short of `need` (and at least 256 bytes)."""
    return torch.empty(max(256, need - 256), dtype=torch.uint8, device="cuda")


def sentinel(n):
    return torch.full((n,), SENTINEL, dtype=torch.int64, device="cuda")


def untouched(t):
    torch.cuda.synchronize()
    return bool((t == SENTINEL).all())


def P(t):
    return ctypes.c_void_p(t.data_ptr())


def stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def count_patterns(gpm):
    return [("3-clique", gpm.clique(3)), ("4-clique", gpm.clique(4)), ("5-clique", gpm.clique(5)),
            ("diamond", gpm.diamond()), ("4-cycle", gpm.cycle4()),
            ("induced 4-path", gpm.pattern(4, [(0, 1), (1, 2), (2, 3)], gpm.VERTEX_INDUCED)),
            ("5-path", gpm.pattern(5, [(0, 1), (1, 2), (2, 3), (3, 4)], gpm.EDGE_INDUCED))]


def test_count_workspace_too_small(gpm, graph):
    lib = gpm.binding.load()
    for name, p in count_patterns(gpm):
        need = gpm.workspace_bytes(graph, p)
        out = sentinel(1)
        ws = small_ws(need)
        rc = lib.gpm_count(graph.handle, ctypes.byref(p), P(ws), ws.numel(), P(out), stream())
        assert rc == OOM, (name, rc)
        assert untouched(out), name
        # the right size works
        assert gpm.count(graph, p) >= 0


def test_list_workspace_too_small(gpm, graph):
    lib = gpm.binding.load()
    for name, p in count_patterns(gpm):
        lp = gpm.binding.Pattern()
        ctypes.pointer(lp)[0] = p
        lp.flags = p.flags | gpm.LIST
        need = gpm.workspace_bytes(graph, lp)
        res = sentinel(3)
        buf = torch.full((64, lp.k), -7, dtype=torch.int32, device="cuda")
        ws = small_ws(need)
        rc = lib.gpm_list(graph.handle, ctypes.byref(lp), P(ws), ws.numel(), P(buf), 64, P(res),
                          stream())
        assert rc == OOM, (name, rc)
        assert untouched(res), name
        assert bool((buf == -7).all()), name


def test_motif_and_fused_workspace_too_small(gpm, graph):
    lib = gpm.binding.load()
    for k in (3, 4):
        out = sentinel(7)
        ws = small_ws(gpm.binding.motif_workspace_bytes(graph, k))
        rc = lib.gpm_motif_count(graph.handle, k, P(ws), ws.numel(), P(out), stream())
        assert rc == OOM, k
        assert untouched(out)
    for k in (3, 4, 5):
        out = sentinel(21)
        ws = small_ws(gpm.motif_enum_workspace_bytes(graph, k))
        rc = lib.gpm_motif_count_enum(graph.handle, k, P(ws), ws.numel(), P(out), stream())
        assert rc == OOM, k
        assert untouched(out)
    out = sentinel(22)
    ws = small_ws(gpm.motif_formula_workspace_bytes(graph, 5))
    rc = lib.gpm_motif_count_formula(graph.handle, 5, P(ws), ws.numel(), P(out), stream())
    assert rc == OOM
    assert untouched(out)
    for kmax in (4, 5):
        out = sentinel(3)
        ws = small_ws(gpm.binding.clique_counts_workspace_bytes(graph, kmax))
        rc = lib.gpm_clique_counts(graph.handle, kmax, P(ws), ws.numel(), P(out), stream())
        assert rc == OOM, kmax
        assert untouched(out)


def test_batch_workspace_too_small(gpm):
    batch = graphgen.rgg_batch(40, seed=3)
    u = torch.from_numpy(batch.u).cuda()
    v = torch.from_numpy(batch.v).cuda()
    g = gpm.Graph.build(batch.n, u, v)
    voff = torch.from_numpy(batch.voff.astype("int32")).cuda()
    lib = gpm.binding.load()
    for k in (3, 4):
        out = sentinel(40 * 7)
        ws = small_ws(gpm.binding.batch_workspace_bytes(40, k))
        rc = lib.gpm_batch_motif_count(g.handle, P(voff), 40, k, P(ws), ws.numel(), P(out),
                                       stream())
        assert rc == OOM, k
        assert untouched(out)
