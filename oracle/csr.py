"""Canonical symmetric CSR from a raw undirected edge stream (numpy).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The input graphs of the method are symmetric, loop-free, free of repeated
edges and have ascending neighbour lists (caption of the input-graph table,
Section 6).  This builds exactly that, the plain way: drop loops, map each
pair to (min, max), keep distinct pairs, emit both directions, sort rows.
"""
import numpy as np


def canonical_csr(n, u, v):
    """Return (off int64[n+1], adj int32[2m]) of the canonical graph."""
    n = int(n)
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    if u.shape != v.shape:
        raise ValueError("u and v differ in length")
    if u.size and (u.min() < 0 or v.min() < 0 or u.max() >= n or v.max() >= n):
        raise ValueError("vertex id out of range")
    keep = u != v
    lo = np.minimum(u[keep], v[keep])
    hi = np.maximum(u[keep], v[keep])
    key = np.unique(lo * max(n, 1) + hi)
    a = key // max(n, 1)
    b = key % max(n, 1)
    rows = np.concatenate([a, b])
    cols = np.concatenate([b, a])
    order = np.lexsort((cols, rows))
    off = np.zeros(n + 1, dtype=np.int64)
    off[1:] = np.cumsum(np.bincount(rows, minlength=n))
    return off, cols[order].astype(np.int32)


def edge_pairs(off, adj):
    """The undirected edges (a < b) of a canonical CSR, ascending."""
    n = off.shape[0] - 1
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(off))
    cols = adj.astype(np.int64)
    m = rows < cols
    return rows[m], cols[m]
