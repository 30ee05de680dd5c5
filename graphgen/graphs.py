"""Synthetic graph generators.

All generators return raw undirected edge streams as two int32 arrays (u, v):
one entry per generated pair, in generation order.  Depending on the
generator the stream may hold self-loops, repeated pairs and both directions
of a pair; turning a stream into a canonical graph is the consumer's job.

Workloads (sizes and parameters):
  * Erdos-Renyi G(n, p): one Bernoulli(p) draw per unordered pair.
  * RMAT (Chakrabarti, Zhan, Faloutsos, SDM 2004) with quadrant
    probabilities (a, b, c, d), sampled bit by bit without noise, Graph500
    style: raw samples are drawn until the stream holds exactly
    ``edge_factor * 2**scale`` distinct undirected non-loop pairs, then every
    vertex id is relabelled by a seeded random permutation.
  * A batch of random geometric graphs in the unit square with a per-graph
    radius chosen for a target mean degree, plus 10% extra uniformly random
    non-edges.
"""
from dataclasses import dataclass
import math

import numpy as np

from .rng import stream_u64, stream_uniform

# stream tags: each generator draws from its own splitmix64 stream(s)
_S_ER = 1
_S_ER_FLIP = 2
_S_RMAT = 3
_S_RMAT_PERM = 4
_S_RGG_N = 5
_S_RGG = 6
_S_RELABEL = 7


@dataclass
class EdgeList:
    """A raw undirected edge stream on vertices 0..n-1."""
    n: int
    u: np.ndarray  # int32[E]
    v: np.ndarray  # int32[E]
    name: str = ""

    @property
    def num_input_edges(self):
        return int(self.u.shape[0])


@dataclass
class BatchEdgeLists:
    """G small graphs; graph g owns vertices voff[g]..voff[g+1]-1 (global ids)
    and stream entries eoff[g]..eoff[g+1]-1."""
    voff: np.ndarray  # int64[G+1]
    eoff: np.ndarray  # int64[G+1]
    u: np.ndarray     # int32[E] global vertex ids
    v: np.ndarray     # int32[E]
    name: str = ""

    @property
    def num_graphs(self):
        return int(self.voff.shape[0] - 1)

    @property
    def n(self):
        return int(self.voff[-1])

    def graph(self, g):
        """Graph g alone, with local vertex ids."""
        lo, hi = int(self.eoff[g]), int(self.eoff[g + 1])
        base = int(self.voff[g])
        return EdgeList(int(self.voff[g + 1] - self.voff[g]),
                        (self.u[lo:hi] - base).astype(np.int32),
                        (self.v[lo:hi] - base).astype(np.int32),
                        name=f"{self.name}[{g}]")


def _as_edges(n, pairs, name):
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    return EdgeList(int(n), pairs[:, 0].astype(np.int32).copy(),
                    pairs[:, 1].astype(np.int32).copy(), name)


# ---------------------------------------------------------------- random ---

def erdos_renyi(n, p, seed):
    """G(n, p): pair {i, j} (i < j) is an edge iff its uniform draw is < p.

    Pairs are visited in row-major order of the strict upper triangle; each
    emitted pair's direction is flipped by one bit of a second stream so the
    stream is not pre-oriented.
    """
    n = int(n)
    iu, ju = np.triu_indices(n, k=1)
    x = stream_uniform(seed, _S_ER, iu.shape[0])
    keep = x < p
    a = iu[keep].astype(np.int32)
    b = ju[keep].astype(np.int32)
    flip = (stream_u64(seed, _S_ER_FLIP, a.shape[0]) & np.uint64(1)).astype(bool)
    u = np.where(flip, b, a).astype(np.int32)
    v = np.where(flip, a, b).astype(np.int32)
    return EdgeList(n, u, v, name=f"er_n{n}_p{p}_s{seed}")


def _rmat_samples(scale, a, b, c, seed, start, count):
    """RMAT samples [start, start+count): 16 random bits per level, four
    levels per u64 word; quadrant thresholds are the cumulative
    probabilities rounded to multiples of 2**-16."""
    words_per = (scale + 3) // 4
    w = stream_u64(seed, _S_RMAT, count * words_per, start * words_per)
    w = w.reshape(count, words_per)
    ta = np.uint64(int(round(a * 65536)))
    tab = np.uint64(int(round((a + b) * 65536)))
    tabc = np.uint64(int(round((a + b + c) * 65536)))
    u = np.zeros(count, dtype=np.int64)
    v = np.zeros(count, dtype=np.int64)
    for lev in range(scale):
        r = (w[:, lev // 4] >> np.uint64(16 * (lev % 4))) & np.uint64(0xFFFF)
        bu = (r >= tab).astype(np.int64)                 # quadrants c, d
        bv = ((r >= ta) & (r < tab)) | (r >= tabc)       # quadrants b, d
        u = (u << 1) | bu
        v = (v << 1) | bv.astype(np.int64)
    return u, v


def rmat(scale, edge_factor=16, a=0.57, b=0.19, c=0.19, seed=20, permute=True):
    """RMAT raw stream holding exactly edge_factor * 2**scale distinct
    undirected non-loop pairs (the stream itself keeps its repeats and loops).
    """
    n = 1 << scale
    target = edge_factor * n
    total = int(target * 1.25) + 1024
    while True:
        u, v = _rmat_samples(scale, a, b, c, seed, 0, total)
        lo = np.minimum(u, v)
        hi = np.maximum(u, v)
        key = lo * n + hi
        key = np.where(u == v, -1, key)
        _, first = np.unique(key, return_index=True)
        first = np.sort(first)
        first = first[key[first] >= 0]
        if first.shape[0] >= target:
            cut = int(first[target - 1]) + 1
            u = u[:cut]
            v = v[:cut]
            break
        total = int(total * 1.5)
    if permute:
        perm = np.argsort(stream_u64(seed, _S_RMAT_PERM, n), kind="stable")
        newid = np.empty(n, dtype=np.int64)
        newid[perm] = np.arange(n, dtype=np.int64)
        u = newid[u]
        v = newid[v]
    return EdgeList(n, u.astype(np.int32), v.astype(np.int32),
                    name=f"rmat{scale}_ef{edge_factor}_s{seed}")


def rgg_batch(num_graphs, seed, nmin=10, nmax=200, deg_lo=3.0, deg_hi=8.0,
              extra_frac=0.1):
    """Batch of random geometric graphs with extra random edges.

    Graph g (independent of num_graphs): n_g uniform in [nmin, nmax]; n_g
    points uniform in the unit square; target mean degree delta uniform in
    [deg_lo, deg_hi]; radius r = sqrt(delta / (pi (n_g - 1))); pair {i, j} is
    an edge iff its squared distance is < r^2.  Then round(extra_frac * m_g)
    uniformly random pairs that are neither loops nor edges yet are added.
    """
    G = int(num_graphs)
    ns = (stream_u64(seed, _S_RGG_N, G) % np.uint64(nmax - nmin + 1)).astype(np.int64) + nmin
    voff = np.zeros(G + 1, dtype=np.int64)
    voff[1:] = np.cumsum(ns)
    us, vs, counts = [], [], []
    for g in range(G):
        ng = int(ns[g])
        # per graph: 2 ng coordinates, 1 degree draw, then extras
        x = stream_uniform(seed, _S_RGG + 16 * g, 2 * ng + 1)
        px, py = x[0:ng], x[ng:2 * ng]
        delta = deg_lo + (deg_hi - deg_lo) * x[2 * ng]
        r2 = delta / (math.pi * (ng - 1))
        iu, ju = np.triu_indices(ng, k=1)
        d2 = (px[iu] - px[ju]) ** 2 + (py[iu] - py[ju]) ** 2
        keep = d2 < r2
        a = iu[keep]
        b = ju[keep]
        m = int(a.shape[0])
        extra = int(math.floor(extra_frac * m + 0.5))
        have = set((a * ng + b).tolist())
        ea, eb = [], []
        pos = 0
        while len(ea) < extra:
            w = stream_u64(seed, _S_RGG + 16 * g + 1, 64, pos)
            pos += 64
            for word in w.tolist():
                i = (word & 0xFFFFFFFF) % ng
                j = (word >> 32) % ng
                if i == j:
                    continue
                lo, hi = (i, j) if i < j else (j, i)
                k = lo * ng + hi
                if k in have:
                    continue
                have.add(k)
                ea.append(lo)
                eb.append(hi)
                if len(ea) == extra:
                    break
        ga = np.concatenate([a, np.asarray(ea, dtype=np.int64)]) + voff[g]
        gb = np.concatenate([b, np.asarray(eb, dtype=np.int64)]) + voff[g]
        us.append(ga)
        vs.append(gb)
        counts.append(ga.shape[0])
    eoff = np.zeros(G + 1, dtype=np.int64)
    eoff[1:] = np.cumsum(counts)
    u = np.concatenate(us).astype(np.int32) if G else np.zeros(0, np.int32)
    v = np.concatenate(vs).astype(np.int32) if G else np.zeros(0, np.int32)
    return BatchEdgeLists(voff, eoff, u, v, name=f"rgg_batch_G{G}_s{seed}")


# ------------------------------------------------------------ structured ---

def complete_graph(n):
    iu, ju = np.triu_indices(int(n), k=1)
    return _as_edges(n, np.stack([iu, ju], 1), f"K{n}")


def star_graph(leaves):
    """Centre 0 joined to leaves 1..leaves."""
    pairs = [(0, i) for i in range(1, leaves + 1)]
    return _as_edges(leaves + 1, pairs, f"star{leaves}")


def cycle_graph(n):
    pairs = [(i, (i + 1) % n) for i in range(n)]
    return _as_edges(n, pairs, f"C{n}")


def path_graph(n):
    pairs = [(i, i + 1) for i in range(n - 1)]
    return _as_edges(n, pairs, f"P{n}")


def complete_bipartite(a, b):
    pairs = [(i, a + j) for i in range(a) for j in range(b)]
    return _as_edges(a + b, pairs, f"K{a},{b}")


def complete_multipartite(parts):
    """Vertices split into consecutive blocks of the given sizes; every pair in
    different blocks is an edge."""
    block = np.repeat(np.arange(len(parts)), parts)
    n = int(block.shape[0])
    iu, ju = np.triu_indices(n, k=1)
    keep = block[iu] != block[ju]
    return _as_edges(n, np.stack([iu[keep], ju[keep]], 1),
                     "K" + ",".join(str(p) for p in parts))


def relabel(g, seed):
    """The same graph under a seeded random vertex permutation."""
    perm = np.argsort(stream_u64(seed, _S_RELABEL, g.n), kind="stable")
    newid = np.empty(g.n, dtype=np.int64)
    newid[perm] = np.arange(g.n, dtype=np.int64)
    return EdgeList(g.n, newid[g.u].astype(np.int32), newid[g.v].astype(np.int32),
                    name=g.name + f"~perm{seed}")


def disjoint_union(graphs):
    """Graphs side by side, ids shifted by the running vertex count."""
    us, vs, base = [], [], 0
    for g in graphs:
        us.append(g.u.astype(np.int64) + base)
        vs.append(g.v.astype(np.int64) + base)
        base += g.n
    u = np.concatenate(us) if us else np.zeros(0)
    v = np.concatenate(vs) if vs else np.zeros(0)
    return EdgeList(base, u.astype(np.int32), v.astype(np.int32),
                    name="+".join(g.name for g in graphs))
