"""CPU oracle for pattern-mining counts and listings.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path never does.  It
shares no code with the device library (its C source is oracle/gpm_oracle.c,
compiled with gcc into oracle/_liboracle.so).

Functions take a canonical CSR from :func:`canonical_csr`.  All counts are
exact Python integers; 128-bit intermediate results from C are recombined
here and must fit in 64 bits where the device path returns uint64.

Parity pins of each function are listed in tests/test_oracle_pins.py.
"""
import ctypes
import os
import subprocess

import numpy as np

from .csr import canonical_csr, edge_pairs

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gpm_oracle.c")
_LIB = os.path.join(_HERE, "_liboracle.so")
_lib = None

MOTIF3_NAMES = ("wedge", "triangle")
MOTIF4_NAMES = ("3-star", "4-path", "4-cycle", "tailed-triangle", "diamond", "4-clique")


def build(force=True):
    """Compile the oracle's C source with gcc (-O2, OpenMP)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11",
                           "-Wall", "-Wextra", "-o", tmp, _SRC])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(_LIB)
        i32, i64, p = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
        u64 = ctypes.c_uint64
        lib.orc_clique_count.argtypes = [i32, p, p, i32, i32, p]
        lib.orc_clique_list.argtypes = [i32, p, p, i32, i32, p, u64, p, p, p]
        lib.orc_edge_triangles.argtypes = [i32, p, p, i32, p]
        lib.orc_motif4_noninduced.argtypes = [i32, p, p, i32, p]
        lib.orc_list_diamonds.argtypes = [i32, p, p, i32, p, u64, p, p, p]
        lib.orc_list_c4.argtypes = [i32, p, p, i32, p, u64, p, p, p]
        lib.orc_wedges.argtypes = [i32, p, p]
        lib.orc_pattern_count.argtypes = [i32, p, p, i32, i32, p, i32, i32, p]
        lib.orc_pattern_count.restype = ctypes.c_int
        lib.orc_pattern_list.argtypes = [i32, p, p, i32, i32, p, i32, p, u64, p, p, p]
        lib.orc_pattern_list.restype = ctypes.c_int
        lib.orc_core_numbers.argtypes = [i32, p, p, p]
        lib.orc_core_numbers.restype = ctypes.c_int
        lib.orc_clique_count_sampled.argtypes = [i32, p, p, i32, i32, i32, i32, p]
        lib.orc_clique_count_sampled.restype = ctypes.c_int
        lib.orc_dag_build.argtypes = [i32, p, p, ctypes.POINTER(ctypes.c_void_p)]
        lib.orc_dag_build.restype = ctypes.c_int
        lib.orc_dag_free.argtypes = [p]
        lib.orc_dag_free.restype = None
        lib.orc_dag_clique_count_sampled.argtypes = [p, i32, i32, i32, i32, p]
        lib.orc_dag_clique_count_sampled.restype = ctypes.c_int
        for f in (lib.orc_clique_count, lib.orc_clique_list, lib.orc_edge_triangles,
                  lib.orc_motif4_noninduced, lib.orc_list_diamonds, lib.orc_list_c4,
                  lib.orc_wedges):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def _prep(off, adj):
    off = np.ascontiguousarray(off, dtype=np.int64)
    adj = np.ascontiguousarray(adj, dtype=np.int32)
    return off, adj, int(off.shape[0] - 1)


def _u128(lo, hi):
    return int(lo) | (int(hi) << 64)


def clique_count(off, adj, k, threads=0):
    """Number of k-cliques (Section 2, problems 1-2)."""
    off, adj, n = _prep(off, adj)
    out = np.zeros(2, dtype=np.uint64)
    _check(_load().orc_clique_count(n, _ptr(off), _ptr(adj), int(k), int(threads), _ptr(out)),
           "clique_count")
    return _u128(out[0], out[1])


def clique_count_sampled(off, adj, k, stride, offset=0, threads=0):
    """k-cliques whose first vertex in the core order has position p with
    p % stride == offset: one share of clique_count's roots.  The shares over
    offset = 0..stride-1 add up to clique_count."""
    off, adj, n = _prep(off, adj)
    out = np.zeros(2, dtype=np.uint64)
    _check(_load().orc_clique_count_sampled(n, _ptr(off), _ptr(adj), int(k), int(threads),
                                            int(stride), int(offset), _ptr(out)),
           "clique_count_sampled")
    return _u128(out[0], out[1])


class CoreDag:
    """The core-ordered DAG of a canonical CSR, built once (the oracle's
    preprocessing), for clique counts rooted at a share of the vertices."""

    def __init__(self, off, adj):
        off, adj, n = _prep(off, adj)
        self._h = ctypes.c_void_p()
        _check(_load().orc_dag_build(n, _ptr(off), _ptr(adj), ctypes.byref(self._h)),
               "dag_build")

    def clique_count_sampled(self, k, stride, offset=0, threads=0):
        """As the module-level clique_count_sampled, on the prebuilt DAG."""
        out = np.zeros(2, dtype=np.uint64)
        _check(_load().orc_dag_clique_count_sampled(self._h, int(k), int(threads), int(stride),
                                                    int(offset), _ptr(out)),
               "dag_clique_count_sampled")
        return _u128(out[0], out[1])

    def close(self):
        if self._h:
            _load().orc_dag_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def triangle_count(off, adj, threads=0):
    return clique_count(off, adj, 3, threads)


def _listing(fn, off, adj, cap, width, *extra):
    off, adj, n = _prep(off, adj)
    buf = np.zeros((max(int(cap), 1), width), dtype=np.int32)
    total = np.zeros(1, dtype=np.uint64)
    written = np.zeros(1, dtype=np.uint64)
    chk = np.zeros(1, dtype=np.uint64)
    _check(fn(n, _ptr(off), _ptr(adj), *extra, _ptr(buf), ctypes.c_uint64(int(cap)),
              _ptr(total), _ptr(written), _ptr(chk)), fn.__name__)
    w = int(written[0])
    return int(total[0]), int(chk[0]), buf[:w].copy()


def clique_list(off, adj, k, cap=0, threads=0):
    """(total, checksum, first `cap` cliques as ascending tuples)."""
    return _listing(_load().orc_clique_list, off, adj, cap, int(k), int(k), int(threads))


def list_diamonds(off, adj, cap=0, threads=0):
    """Edge-induced diamonds: (total, checksum, rows (a, b, c, d)), a-b the diagonal."""
    return _listing(_load().orc_list_diamonds, off, adj, cap, 4, int(threads))


def list_c4(off, adj, cap=0, threads=0):
    """Edge-induced 4-cycles: (total, checksum, rows (v0, v1, v2, v3) in cycle order)."""
    return _listing(_load().orc_list_c4, off, adj, cap, 4, int(threads))


def edge_triangles(off, adj, threads=0):
    """T per arc of the symmetric CSR: |N(x) ∩ N(y)| (Section 5, local counting)."""
    off, adj, n = _prep(off, adj)
    te = np.zeros(max(int(off[-1]), 1), dtype=np.int64)
    _check(_load().orc_edge_triangles(n, _ptr(off), _ptr(adj), int(threads), _ptr(te)),
           "edge_triangles")
    return te[: int(off[-1])]


def motif4_noninduced(off, adj, threads=0):
    """Non-induced copies of the six connected 4-vertex patterns, in the order
    3-star, 4-path, 4-cycle, tailed-triangle, diamond, 4-clique."""
    off, adj, n = _prep(off, adj)
    out = np.zeros(12, dtype=np.uint64)
    _check(_load().orc_motif4_noninduced(n, _ptr(off), _ptr(adj), int(threads), _ptr(out)),
           "motif4_noninduced")
    return [_u128(out[2 * i], out[2 * i + 1]) for i in range(6)]


def wedge_sum(off):
    """sum_v C(d_v, 2)."""
    off = np.ascontiguousarray(off, dtype=np.int64)
    out = np.zeros(2, dtype=np.uint64)
    _check(_load().orc_wedges(int(off.shape[0] - 1), _ptr(off), _ptr(out)), "wedges")
    return _u128(out[0], out[1])


def motif3(off, adj, threads=0):
    """Induced 3-motif counts [wedge, triangle].  Triangles by clique counting;
    open wedges = sum_v C(d_v, 2) - 3T, each triangle closing three wedges
    (3-motif local-counting listing, Appendix A)."""
    t = triangle_count(off, adj, threads)
    return [wedge_sum(off) - 3 * t, t]


def motif4(off, adj, threads=0):
    """Induced 4-motif counts [3-star, 4-path, 4-cycle, tailed-triangle,
    diamond, 4-clique] from non-induced counts N by back-substitution
    N = M I, M[P][H] = copies of P spanning H:
      K4: 1 -> itself; diamond: 6 in K4; paw: 4 per diamond, 12 per K4;
      4-cycle: 1 per diamond, 3 per K4; 4-path: 2 per paw, 4 per 4-cycle,
      6 per diamond, 12 per K4; 3-star: 1 per paw, 2 per diamond, 4 per K4.
    """
    claw, p4, c4, paw, dia, k4 = motif4_noninduced(off, adj, threads)
    i_k4 = k4
    i_dia = dia - 6 * i_k4
    i_paw = paw - 4 * i_dia - 12 * i_k4
    i_c4 = c4 - i_dia - 3 * i_k4
    i_p4 = p4 - 2 * i_paw - 4 * i_c4 - 6 * i_dia - 12 * i_k4
    i_claw = claw - i_paw - 2 * i_dia - 4 * i_k4
    res = [i_claw, i_p4, i_c4, i_paw, i_dia, i_k4]
    if min(res) < 0:
        raise AssertionError(f"negative induced count {res}")
    return res


def batch_motifs(batch, k, threads=1):
    """Per-graph induced k-motif counts (k = 3 or 4) for a BatchEdgeLists."""
    out = []
    for g in range(batch.num_graphs):
        e = batch.graph(g)
        off, adj = canonical_csr(e.n, e.u, e.v)
        out.append(motif3(off, adj, threads) if k == 3 else motif4(off, adj, threads))
    return out


def pattern_list(off, adj, k, edges, induced, cap=0):
    """Embeddings of a connected pattern, each once: (total, checksum, rows)
    with row i = the data vertices of pattern vertices 0..k-1, the
    representative being the lexicographically smallest of the embedding's
    automorphic maps.  Checksum key: the ascending vertex tuple
    (vertex-induced) or the ascending edge codes (edge-induced)."""
    pe = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1))
    return _listing(_load().orc_pattern_list, off, adj, cap, int(k), int(k),
                    int(pe.shape[0] // 2), _ptr(pe), int(bool(induced)))


def core_numbers(off, adj):
    """Core number of every vertex (the core values of Appendix B.2's
    core-based orientation): by bucket peeling, a vertex's remaining degree
    when it is removed."""
    off, adj, n = _prep(off, adj)
    out = np.zeros(max(n, 1), dtype=np.int32)
    _check(_load().orc_core_numbers(n, _ptr(off), _ptr(adj), _ptr(out)), "core_numbers")
    return out[:n]


def pattern_count(off, adj, k, edges, induced, threads=0):
    """Embeddings of the connected pattern with k vertices and the given
    edge list (pairs of pattern vertices): vertex-induced (motif counting)
    or edge-induced (subgraph listing), Section 2's problem definitions.
    Plain definition: injective maps onto edges (and non-edges when
    induced) counted by backtracking, divided by the pattern's automorphism
    count.  Returns (count, automorphisms)."""
    off, adj, n = _prep(off, adj)
    pe = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1))
    out = np.zeros(3, dtype=np.uint64)
    _check(_load().orc_pattern_count(n, _ptr(off), _ptr(adj), int(k), int(pe.shape[0] // 2),
                                     _ptr(pe), int(bool(induced)), int(threads), _ptr(out)),
           "pattern_count")
    return _u128(out[0], out[1]), int(out[2])
