"""ctypes binding of include/gpm.h (same names, argument marshalling only)."""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgpmhip.so")

VERTEX_INDUCED = 0x1
EDGE_INDUCED = 0x2
LIST = 0x4

ORIENT_DEGREE = 1
ORIENT_CORE = 2
MOTIF3_NAMES = ("wedge", "triangle")
MOTIF4_NAMES = ("3-star", "4-path", "4-cycle", "tailed-triangle", "diamond", "4-clique")

_STATUS = {0: "GPM_OK", 1: "GPM_INVALID_ARGUMENT", 2: "GPM_OUT_OF_MEMORY",
           3: "GPM_DEVICE_ERROR", 4: "GPM_TRUNCATED", 5: "GPM_UNSUPPORTED",
           6: "GPM_NOT_CANONICAL", 7: "GPM_INCONSISTENT"}


class GpmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Pattern(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("n_edges", ctypes.c_int32),
                ("edges", (ctypes.c_int32 * 2) * 36), ("flags", ctypes.c_uint32)]


class Tuning(ctypes.Structure):
    """gpm_tuning: task granularity of the plain path (per graph handle)."""
    _fields_ = [("tc_tau", ctypes.c_int64 * 3), ("tc_blocks_per_cu", ctypes.c_int32 * 3),
                ("clique_wave_blocks_per_cu", ctypes.c_int32), ("lg5_slice", ctypes.c_int64)]

    def as_dict(self):
        return {"tc_tau": list(self.tc_tau), "tc_blocks_per_cu": list(self.tc_blocks_per_cu),
                "clique_wave_blocks_per_cu": int(self.clique_wave_blocks_per_cu),
                "lg5_slice": int(self.lg5_slice)}


class _GraphInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("max_degree", ctypes.c_int32),
                ("m", ctypes.c_int64), ("max_out_degree", ctypes.c_int32),
                ("reserved", ctypes.c_int32),
                ("off", ctypes.c_void_p), ("adj", ctypes.c_void_p),
                ("dag_off", ctypes.c_void_p), ("dag_adj", ctypes.c_void_p),
                ("dag_src", ctypes.c_void_p)]


_lib = None


def library_path():
    return _LIB_PATH


def load():
    """Loads libgpmhip.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with "
                          "python -m paper_2011_03135_amd.build")
    lib = ctypes.CDLL(_LIB_PATH)
    P, i32, i64, u32, u64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                             ctypes.c_uint32, ctypes.c_uint64)
    sigs = {
        "gpm_status_string": ([i32], ctypes.c_char_p),
        "gpm_last_error": ([], ctypes.c_char_p),
        "gpm_version": ([], ctypes.c_char_p),
        "gpm_pattern_from_edges": ([i32, i32, P, u32, P], i32),
        "gpm_pattern_clique": ([i32, u32, P], i32),
        "gpm_pattern_plan": ([P, P], i32),
        "gpm_pattern_matching_order": ([P, P, P], i32),
        "gpm_graph_build_bytes": ([i32, i64, P, P], i32),
        "gpm_graph_build": ([i32, P, P, i64, P, u64, P, u64, P, P], i32),
        "gpm_graph_from_csr_bytes": ([i32, i64, P, P], i32),
        "gpm_graph_from_csr": ([i32, P, P, i64, i32, P, u64, P, u64, P, P], i32),
        "gpm_graph_get_info": ([P, P], i32),
        "gpm_graph_release": ([P], None),
        "gpm_workspace_bytes": ([P, P, P], i32),
        "gpm_count": ([P, P, P, u64, P, P], i32),
        "gpm_list": ([P, P, P, u64, P, u64, P, P], i32),
        "gpm_clique_counts_workspace_bytes": ([P, i32, P], i32),
        "gpm_clique_counts": ([P, i32, P, u64, P, P], i32),
        "gpm_motif_workspace_bytes": ([P, i32, P], i32),
        "gpm_motif_count": ([P, i32, P, u64, P, P], i32),
        "gpm_graph_orient_bytes": ([P, P], i32),
        "gpm_graph_orient": ([P, i32, P, u64, P, P], i32),
        "gpm_graph_get_tuning": ([P, P], i32),
        "gpm_graph_set_tuning": ([P, P], i32),
        "gpm_graph_autotune_bytes": ([P, P], i32),
        "gpm_graph_autotune": ([P, P, u64, P, P], i32),
        "gpm_motif_classes": ([i32], i32),
        "gpm_motif_class_pattern": ([i32, i32, P], i32),
        "gpm_motif_enum_workspace_bytes": ([P, i32, P], i32),
        "gpm_motif_count_enum": ([P, i32, P, u64, P, P], i32),
        "gpm_motif_formula_workspace_bytes": ([P, i32, P], i32),
        "gpm_motif_count_formula": ([P, i32, P, u64, P, P], i32),
        "gpm_batch_workspace_bytes": ([i32, i32, P], i32),
        "gpm_batch_motif_count": ([P, P, i32, i32, P, u64, P, P], i32),
        "gpm_batch_default_config": ([P], i32),
        "gpm_batch_motif_count_config": ([P, P, i32, i32, P, P, u64, P, P], i32),
        "gpm_batch_autotune": ([P, P, i32, i32, P, u64, P, P, i32, P, P], i32),
        "gpm_batch_motif_count_static": ([P, P, i32, i32, P, P], i32),
        "gpm_timing_enable": ([i32], i32),
        "gpm_timing_read": ([P, P, P, i32], i32),
        "gpm_server_create": ([P, P], i32),
        "gpm_server_submit": ([P, P, P], i32),
        "gpm_server_poll": ([P, P, i32, P], i32),
        "gpm_server_pending": ([P], i64),
        "gpm_server_now": ([], ctypes.c_double),
        "gpm_server_destroy": ([P], None),
    }
    for name, (args, res) in sigs.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _check(rc):
    if rc != 0:
        msg = load().gpm_last_error().decode(errors="replace")
        raise GpmError(rc, msg)


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _buffer(nbytes, device):
    t = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
    if t.data_ptr() % 256:
        raise GpmError(1, "allocator returned a buffer that is not 256-byte aligned")
    return t


def _u64(x):
    x = int(x)
    return x + (1 << 64) if x < 0 else x


def pattern(k, edges, flags):
    """gpm_pattern_from_edges: edges is a list of (a, b) pairs on 0..k-1."""
    lib = load()
    flat = (ctypes.c_int32 * (2 * max(len(edges), 1)))(*[x for e in edges for x in e])
    p = Pattern()
    _check(lib.gpm_pattern_from_edges(int(k), len(edges), flat, int(flags), ctypes.byref(p)))
    return p


def matching_order(p):
    """gpm_pattern_matching_order -> (order, less): the general plan's
    matching order (pattern vertex per step) and its partial orders, less[x]
    = the set of pattern vertices y with f(x) < f(y) required."""
    order = (ctypes.c_int32 * 9)()
    less = (ctypes.c_uint32 * 9)()
    _check(load().gpm_pattern_matching_order(ctypes.byref(p), order, less))
    return ([order[i] for i in range(p.k)],
            [{y for y in range(p.k) if (less[x] >> y) & 1} for x in range(p.k)])


def clique(k, flags=VERTEX_INDUCED):
    p = Pattern()
    _check(load().gpm_pattern_clique(int(k), int(flags), ctypes.byref(p)))
    return p


def diamond(flags=EDGE_INDUCED):
    """Diamond with diagonal (0, 1) and tips 2, 3."""
    return pattern(4, [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3)], flags)


def cycle4(flags=EDGE_INDUCED):
    """4-cycle 0-1-2-3-0."""
    return pattern(4, [(0, 1), (1, 2), (2, 3), (3, 0)], flags)


class Graph:
    """A canonical, degree-oriented graph in caller-owned (torch) device memory."""

    def __init__(self, handle, storage, device):
        self._h = handle
        self._storage = storage
        self.device = device
        info = _GraphInfo()
        _check(load().gpm_graph_get_info(self._h, ctypes.byref(info)))
        self.n = info.n
        self.m = info.m
        self.max_degree = info.max_degree
        self.max_out_degree = info.max_out_degree
        self._info = info

    @staticmethod
    def build_bytes(n, n_input_edges):
        gb, sb = ctypes.c_uint64(), ctypes.c_uint64()
        _check(load().gpm_graph_build_bytes(int(n), int(n_input_edges), ctypes.byref(gb),
                                            ctypes.byref(sb)))
        return gb.value, sb.value

    @classmethod
    def build(cls, n, u, v, stream=None, scratch=None, storage=None):
        """gpm_graph_build from int32 CUDA tensors u, v (a raw edge stream).
        storage / scratch: optional preallocated uint8 device buffers."""
        if u.dtype != torch.int32 or v.dtype != torch.int32 or not u.is_cuda or not v.is_cuda:
            raise TypeError("u and v must be int32 CUDA tensors")
        if u.shape != v.shape or u.dim() != 1:
            raise ValueError("u and v must be 1-D of equal length")
        u = u.contiguous()
        v = v.contiguous()
        gb, sb = cls.build_bytes(n, u.shape[0])
        if storage is None or storage.numel() < gb:
            storage = _buffer(gb, u.device)
        if scratch is None or scratch.numel() < sb:
            scratch = _buffer(sb, u.device)
        h = ctypes.c_void_p()
        _check(load().gpm_graph_build(int(n), _ptr(u), _ptr(v), int(u.shape[0]), _ptr(storage),
                                      gb, _ptr(scratch), sb, _stream(stream), ctypes.byref(h)))
        return cls(h, storage, u.device)

    @staticmethod
    def from_csr_bytes(n, nnz):
        gb, sb = ctypes.c_uint64(), ctypes.c_uint64()
        _check(load().gpm_graph_from_csr_bytes(int(n), int(nnz), ctypes.byref(gb),
                                               ctypes.byref(sb)))
        return gb.value, sb.value

    @classmethod
    def from_csr(cls, n, off, adj, validate=True, stream=None, scratch=None, storage=None):
        """gpm_graph_from_csr from int32 CUDA tensors off [n+1] and adj [nnz]
        holding a symmetric CSR in canonical form (checked when validate)."""
        for t in (off, adj):
            if t.dtype != torch.int32 or not t.is_cuda or t.dim() != 1:
                raise TypeError("off and adj must be 1-D int32 CUDA tensors")
        if off.shape[0] != int(n) + 1:
            raise ValueError("off must have n + 1 entries")
        off = off.contiguous()
        adj = adj.contiguous()
        gb, sb = cls.from_csr_bytes(n, adj.shape[0])
        if storage is None or storage.numel() < gb:
            storage = _buffer(gb, off.device)
        if scratch is None or scratch.numel() < sb:
            scratch = _buffer(sb, off.device)
        h = ctypes.c_void_p()
        _check(load().gpm_graph_from_csr(int(n), _ptr(off), _ptr(adj), int(adj.shape[0]),
                                         1 if validate else 0, _ptr(storage), gb, _ptr(scratch),
                                         sb, _stream(stream), ctypes.byref(h)))
        return cls(h, storage, off.device)

    def orient(self, order, stream=None, scratch=None, core_out=None):
        """gpm_graph_orient: rebuild the DAG by degree (ORIENT_DEGREE) or by
        core value (ORIENT_CORE); returns the core numbers (int32 device
        tensor) when core_out is True or a tensor to fill, else None."""
        nb = ctypes.c_uint64()
        _check(load().gpm_graph_orient_bytes(self._h, ctypes.byref(nb)))
        if scratch is None or scratch.numel() < nb.value:
            scratch = _buffer(nb.value, self.device)
        core = None
        if core_out is True:
            core = torch.empty(max(self.n, 1), dtype=torch.int32, device=self.device)
        elif core_out is not None and core_out is not False:
            core = core_out
        _check(load().gpm_graph_orient(self._h, int(order), _ptr(scratch), scratch.numel(),
                                       _ptr(core) if core is not None else None,
                                       _stream(stream)))
        info = _GraphInfo()
        _check(load().gpm_graph_get_info(self._h, ctypes.byref(info)))
        self.max_out_degree = info.max_out_degree
        self._info = info
        return core[:self.n] if core is not None else None

    def tuning(self):
        """gpm_graph_get_tuning -> dict (tc_tau, tc_blocks_per_cu,
        clique_wave_blocks_per_cu, lg5_slice)."""
        t = Tuning()
        _check(load().gpm_graph_get_tuning(self._h, ctypes.byref(t)))
        return t.as_dict()

    def set_tuning(self, tc_tau=None, tc_blocks_per_cu=None, clique_wave_blocks_per_cu=None,
                   lg5_slice=None):
        """gpm_graph_set_tuning; unnamed knobs keep their values."""
        t = Tuning()
        _check(load().gpm_graph_get_tuning(self._h, ctypes.byref(t)))
        if tc_tau is not None:
            t.tc_tau = (ctypes.c_int64 * 3)(*[int(x) for x in tc_tau])
        if tc_blocks_per_cu is not None:
            t.tc_blocks_per_cu = (ctypes.c_int32 * 3)(*[int(x) for x in tc_blocks_per_cu])
        if clique_wave_blocks_per_cu is not None:
            t.clique_wave_blocks_per_cu = int(clique_wave_blocks_per_cu)
        if lg5_slice is not None:
            t.lg5_slice = int(lg5_slice)
        _check(load().gpm_graph_set_tuning(self._h, ctypes.byref(t)))

    def autotune(self, stream=None, ws=None):
        """gpm_graph_autotune: picks the tuning for this graph by timing it;
        returns the chosen tuning (dict)."""
        nb = ctypes.c_uint64()
        _check(load().gpm_graph_autotune_bytes(self._h, ctypes.byref(nb)))
        if ws is None or ws.numel() < nb.value:
            ws = _buffer(nb.value, self.device)
        t = Tuning()
        _check(load().gpm_graph_autotune(self._h, _ptr(ws), ws.numel(), _stream(stream),
                                         ctypes.byref(t)))
        return t.as_dict()

    def csr(self):
        """(off, adj) views (int32 device tensors) of the symmetric CSR."""
        return self._view(self._info.off, self.n + 1), self._view(self._info.adj, 2 * self.m)

    def dag(self):
        """(dag_off, dag_adj, dag_src) views of the oriented CSR."""
        return (self._view(self._info.dag_off, self.n + 1),
                self._view(self._info.dag_adj, self.m), self._view(self._info.dag_src, self.m))

    def _view(self, addr, count):
        base = self._storage.data_ptr()
        start = (addr - base) // 4
        return self._storage.view(torch.int32)[start:start + int(count)]

    @property
    def handle(self):
        return self._h

    def __del__(self):
        try:
            if self._h:
                load().gpm_graph_release(self._h)
                self._h = None
        except Exception:
            pass


def timing_enable(on=True):
    """gpm_timing_enable: bracket the library's main kernels with HIP events."""
    _check(load().gpm_timing_enable(1 if on else 0))


def timing_read(cap=4096):
    """gpm_timing_read -> list of (kernel name, milliseconds, work units)."""
    names = (ctypes.c_char_p * cap)()
    ms = (ctypes.c_float * cap)()
    units = (ctypes.c_uint64 * cap)()
    k = load().gpm_timing_read(names, ms, units, cap)
    return [(names[i].decode(), float(ms[i]), int(units[i])) for i in range(min(k, cap))]


def workspace_bytes(g, p):
    b = ctypes.c_uint64()
    _check(load().gpm_workspace_bytes(g.handle, ctypes.byref(p), ctypes.byref(b)))
    return b.value


def count(g, p, stream=None, ws=None, out=None):
    """gpm_count -> exact int (synchronises the stream when out is None)."""
    nb = workspace_bytes(g, p)
    if ws is None or ws.numel() < nb:
        ws = _buffer(nb, g.device)
    res = out if out is not None else torch.zeros(1, dtype=torch.int64, device=g.device)
    _check(load().gpm_count(g.handle, ctypes.byref(p), _ptr(ws), ws.numel(), _ptr(res),
                            _stream(stream)))
    if out is not None:
        return out
    return _u64(res.item())


def list_embeddings(g, p, cap, stream=None, ws=None):
    """gpm_list -> (total, written, checksum, rows[written, k] int32 tensor)."""
    nb = workspace_bytes(g, p)
    if ws is None or ws.numel() < nb:
        ws = _buffer(nb, g.device)
    k = p.k
    buf = torch.empty((max(int(cap), 1), k), dtype=torch.int32, device=g.device)
    res = torch.zeros(3, dtype=torch.int64, device=g.device)
    _check(load().gpm_list(g.handle, ctypes.byref(p), _ptr(ws), ws.numel(), _ptr(buf), int(cap),
                           _ptr(res), _stream(stream)))
    total, written, chk = (_u64(x) for x in res.tolist())
    return total, written, chk, buf[:written]


def clique_counts_workspace_bytes(g, kmax):
    b = ctypes.c_uint64()
    _check(load().gpm_clique_counts_workspace_bytes(g.handle, int(kmax), ctypes.byref(b)))
    return b.value


def clique_counts(g, kmax, stream=None, ws=None, out=None):
    """gpm_clique_counts: [3-cliques, ..., kmax-cliques] from one pass.  With
    `out` (int64 device tensor of kmax - 2 entries) the call only enqueues
    and returns `out`; otherwise it waits and returns Python ints."""
    need = clique_counts_workspace_bytes(g, kmax)
    if ws is None:
        ws = _buffer(need, g.device)
    elif ws.numel() < need:
        raise GpmError(2, f"workspace of {ws.numel()} bytes, {need} needed")
    res = out if out is not None else torch.zeros(int(kmax) - 2, dtype=torch.int64,
                                                  device=g.device)
    _check(load().gpm_clique_counts(g.handle, int(kmax), _ptr(ws), ws.numel(), _ptr(res),
                                    _stream(stream)))
    if out is not None:
        return out
    return [_u64(x) for x in res.tolist()]


def motif_workspace_bytes(g, k):
    b = ctypes.c_uint64()
    _check(load().gpm_motif_workspace_bytes(g.handle, int(k), ctypes.byref(b)))
    return b.value


def motif_count(g, k, stream=None, ws=None, out=None):
    """gpm_motif_count -> list of exact ints (3-motifs: 2, 4-motifs: 6)."""
    b = ctypes.c_uint64()
    _check(load().gpm_motif_workspace_bytes(g.handle, int(k), ctypes.byref(b)))
    if ws is None or ws.numel() < b.value:
        ws = _buffer(b.value, g.device)
    nout = 3 if k == 3 else 7
    res = out if out is not None else torch.zeros(nout, dtype=torch.int64, device=g.device)
    _check(load().gpm_motif_count(g.handle, int(k), _ptr(ws), ws.numel(), _ptr(res),
                                  _stream(stream)))
    if out is not None:
        return out
    vals = [_u64(x) for x in res.tolist()]
    if vals[-1] != 0:
        raise GpmError(7, f"motif combination check failed (status word {vals[-1]})")
    return vals[:-1]


def motif_classes(k):
    """gpm_motif_classes: number of k-vertex motif classes (0 if k is unsupported)."""
    return int(load().gpm_motif_classes(int(k)))


def motif_class_pattern(k, index):
    """gpm_motif_class_pattern -> list of the class's edges (a, b), a < b."""
    p = Pattern()
    _check(load().gpm_motif_class_pattern(int(k), int(index), ctypes.byref(p)))
    return [(p.edges[i][0], p.edges[i][1]) for i in range(p.n_edges)]


def motif_enum_workspace_bytes(g, k):
    b = ctypes.c_uint64()
    _check(load().gpm_motif_enum_workspace_bytes(g.handle, int(k), ctypes.byref(b)))
    return b.value


def motif_count_enum(g, k, stream=None, ws=None, out=None):
    """gpm_motif_count_enum -> list of exact ints, one per motif class."""
    nbytes = motif_enum_workspace_bytes(g, k)
    if ws is None or ws.numel() < nbytes:
        ws = _buffer(nbytes, g.device)
    nout = motif_classes(k)
    res = out if out is not None else torch.zeros(nout, dtype=torch.int64, device=g.device)
    _check(load().gpm_motif_count_enum(g.handle, int(k), _ptr(ws), ws.numel(), _ptr(res),
                                       _stream(stream)))
    if out is not None:
        return out
    return [_u64(x) for x in res.tolist()]


def motif_formula_workspace_bytes(g, k=5):
    b = ctypes.c_uint64()
    _check(load().gpm_motif_formula_workspace_bytes(g.handle, int(k), ctypes.byref(b)))
    return b.value


def motif_count_formula(g, k=5, stream=None, ws=None, out=None):
    """gpm_motif_count_formula -> the 21 induced 5-motif counts (exact ints),
    by local-count formulas and back-substitution.  With `out` (int64 device
    tensor of 22 entries) the call only enqueues and returns `out`."""
    nbytes = motif_formula_workspace_bytes(g, k)
    if ws is None or ws.numel() < nbytes:
        ws = _buffer(nbytes, g.device)
    res = out if out is not None else torch.zeros(22, dtype=torch.int64, device=g.device)
    _check(load().gpm_motif_count_formula(g.handle, int(k), _ptr(ws), ws.numel(), _ptr(res),
                                          _stream(stream)))
    if out is not None:
        return out
    vals = [_u64(x) for x in res.tolist()]
    if vals[-1] != 0:
        raise GpmError(7, f"formula check failed (status word {vals[-1]})")
    return vals[:-1]


class BatchConfig(ctypes.Structure):
    """gpm_batch_config: team_threads, tiers, blocks_per_cu."""
    _fields_ = [("team_threads", ctypes.c_int32), ("tiers", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {"team_threads": self.team_threads, "tiers": self.tiers,
                "blocks_per_cu": self.blocks_per_cu}


def batch_default_config():
    c = BatchConfig()
    _check(load().gpm_batch_default_config(ctypes.byref(c)))
    return c


def batch_workspace_bytes(G, k):
    b = ctypes.c_uint64()
    _check(load().gpm_batch_workspace_bytes(int(G), int(k), ctypes.byref(b)))
    return b.value


def _batch_args(g, voff, k, ws, out):
    G = int(voff.shape[0] - 1)
    if voff.dtype != torch.int32 or not voff.is_cuda:
        raise TypeError("voff must be an int32 CUDA tensor")
    need = batch_workspace_bytes(G, k)
    if ws is None:
        ws = _buffer(need, g.device)
    elif ws.numel() < need:
        raise GpmError(2, f"batch workspace of {ws.numel()} bytes, {need} needed")
    width = 3 if k == 3 else 7
    res = out if out is not None else torch.zeros((G, width), dtype=torch.int64, device=g.device)
    return G, ws, res


def batch_motif_count(g, voff, k, stream=None, ws=None, out=None, config=None):
    """gpm_batch_motif_count (or _config when `config` is given) -> int64
    tensor [G, 3 or 7] (uint64 bits)."""
    G, ws, res = _batch_args(g, voff, k, ws, out)
    if config is None:
        _check(load().gpm_batch_motif_count(g.handle, _ptr(voff.contiguous()), G, int(k),
                                            _ptr(ws), ws.numel(), _ptr(res), _stream(stream)))
    else:
        _check(load().gpm_batch_motif_count_config(g.handle, _ptr(voff.contiguous()), G, int(k),
                                                   ctypes.byref(config), _ptr(ws), ws.numel(),
                                                   _ptr(res), _stream(stream)))
    return res


BATCH_STATIC_SCRATCH_BYTES = 4 << 20
BATCH_STATIC_MAX_GRAPHS = 1045492


def batch_motif_count_static(g, voff, k, stream=None, out=None):
    """gpm_batch_motif_count_static: the batch's work area in the library's
    static device scratch (no workspace argument, nothing allocated by the
    library) -> int64 tensor [G, 3 or 7] (uint64 bits)."""
    G = int(voff.shape[0] - 1)
    if voff.dtype != torch.int32 or not voff.is_cuda:
        raise TypeError("voff must be an int32 CUDA tensor")
    width = 3 if k == 3 else 7
    res = out if out is not None else torch.zeros((G, width), dtype=torch.int64, device=g.device)
    _check(load().gpm_batch_motif_count_static(g.handle, _ptr(voff.contiguous()), G, int(k),
                                               _ptr(res), _stream(stream)))
    return res


def batch_autotune(g, voff, k, reps=3, stream=None, ws=None, out=None):
    """gpm_batch_autotune -> (BatchConfig, mean ms per call, counts tensor)."""
    G, ws, res = _batch_args(g, voff, k, ws, out)
    best = BatchConfig()
    ms = ctypes.c_float()
    _check(load().gpm_batch_autotune(g.handle, _ptr(voff.contiguous()), G, int(k), _ptr(ws),
                                     ws.numel(), _ptr(res), _stream(stream), int(reps),
                                     ctypes.byref(best), ctypes.byref(ms)))
    return best, ms.value, res


# ------------------------------------------------------------- serving ---

QUERY_CLIQUE = 1
QUERY_MOTIF = 2


class _ServerConfig(ctypes.Structure):
    _fields_ = [("max_slots", ctypes.c_int32), ("cu_percent", ctypes.c_int32),
                ("d_pool", ctypes.c_void_p), ("pool_bytes", ctypes.c_uint64)]


class _Request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("k", ctypes.c_int32),
                ("graph", ctypes.c_void_p), ("tag", ctypes.c_uint64)]


class Response(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("tag", ctypes.c_uint64),
                ("status", ctypes.c_int32), ("n_values", ctypes.c_int32),
                ("values", ctypes.c_uint64 * 7),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double),
                ("d_start", ctypes.c_double), ("d_end", ctypes.c_double)]

    def counts(self):
        return [int(self.values[i]) for i in range(self.n_values)]


class Server:
    """gpm_server_*: concurrent request execution over resident graphs."""

    def __init__(self, max_slots=4, pool_bytes=8 << 30, device="cuda", cu_percent=0):
        self._pool = _buffer(pool_bytes, torch.device(device))
        cfg = _ServerConfig(int(max_slots), int(cu_percent), self._pool.data_ptr(),
                            int(self._pool.numel()))
        self._h = ctypes.c_void_p()
        _check(load().gpm_server_create(ctypes.byref(cfg), ctypes.byref(self._h)))
        self._graphs = {}

    def submit(self, graph, kind, k, tag=0):
        req = _Request(int(kind), int(k), graph.handle, int(tag))
        rid = ctypes.c_uint64()
        _check(load().gpm_server_submit(self._h, ctypes.byref(req), ctypes.byref(rid)))
        self._graphs[rid.value] = graph     # keep the graph alive while in flight
        return rid.value

    def poll(self, max_n=1024):
        buf = (Response * max_n)()
        n = ctypes.c_int32()
        _check(load().gpm_server_poll(self._h, buf, max_n, ctypes.byref(n)))
        out = [buf[i] for i in range(n.value)]
        for r in out:
            self._graphs.pop(r.id, None)
        return out

    def pending(self):
        return int(load().gpm_server_pending(self._h))

    @staticmethod
    def now():
        return float(load().gpm_server_now())

    def close(self):
        if self._h:
            load().gpm_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
