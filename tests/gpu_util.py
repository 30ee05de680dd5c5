"""Helpers shared by the GPU tests: upload a raw edge stream and build."""
import numpy as np
import torch


def upload(e):
    u = torch.from_numpy(np.ascontiguousarray(e.u, dtype=np.int32)).cuda()
    v = torch.from_numpy(np.ascontiguousarray(e.v, dtype=np.int32)).cuda()
    return u, v


def build(gpm, e):
    u, v = upload(e)
    return gpm.Graph.build(e.n, u, v)


def degree_rank_dag(off, adj):
    """Arcs (a, b) of the degree-ordered DAG from a canonical CSR (numpy)."""
    n = off.shape[0] - 1
    deg = np.diff(off).astype(np.int64)
    rows = np.repeat(np.arange(n, dtype=np.int64), deg)
    cols = adj.astype(np.int64)
    keep = (deg[rows] < deg[cols]) | ((deg[rows] == deg[cols]) & (rows < cols))
    return rows[keep], cols[keep]
