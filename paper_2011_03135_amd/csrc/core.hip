// Core numbers and the core-value orientation (Appendix B.2 names two
// orientations for cliques: by degree and by core value).
//
// Core numbers by level-synchronous peeling.  For level L = 0, 1, ...: every
// vertex not yet removed whose remaining degree is at most L is removed with
// core number L (a scan over the vertices), and removing a vertex lowers
// its live neighbours' remaining degrees (atomic decrements); a neighbour
// whose degree falls from L + 1 to L is removed at the same level, in the
// next sub-round.  Each vertex is removed once, when the decrement that
// takes it to L is the one that sees L + 1, so the frontier lists never
// repeat a vertex.  Levels with nothing to remove are skipped by taking the
// smallest remaining degree.  The host drives the levels and reads one
// counter per sub-round.
//
// Orientation: arc u -> v iff (key(u), u) < (key(v), v); each row's arcs
// keep ascending id order.  By degree, key = the degree (the build's
// orientation).  By core value, key = (core << S) | min(degree, 2^S - 1),
// S = 31 - bits(largest core): the core value first, then, among equal core
// values, the degree, so a hub does not point at its whole core (by core
// value and id alone, RMAT-20's largest out-degree is 1289; with the degree
// as second key 702, against 707 by degree and 639 for the degeneracy).
#include <algorithm>
#include <climits>

#include "gpm_internal.h"

namespace gpm {

namespace {

constexpr int kCoreBlock = 256;
constexpr int kCoreWaves = kCoreBlock / kWave;

// ctl words
enum { C_MIN_DEG = 0, C_LIVE = 1, C_CNT0 = 2, C_CNT1 = 3, C_MAX_OUT = 4, C_WORDS = 8 };

__global__ void __launch_bounds__(kCoreBlock) k_core_init(const int32_t *__restrict__ off,
                                                          int32_t n, int32_t *deg,
                                                          int32_t *core) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        deg[v] = off[v + 1] - off[v];
        core[v] = -1;
    }
}

// ctl[C_MIN_DEG] = smallest remaining degree, ctl[C_LIVE] = vertices left.
__global__ void __launch_bounds__(kCoreBlock) k_core_stats(int32_t n, const int32_t *deg,
                                                           const int32_t *core, uint32_t *ctl) {
    int32_t mn = INT_MAX, live = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        if (core[v] < 0) {
            mn = min(mn, deg[v]);
            live++;
        }
    }
    mn = -wave_max(-mn);
    live = wave_sum(live);
    if (lane_id() == 0 && live > 0) {
        atomicMin(ctl + C_MIN_DEG, (uint32_t)mn);
        atomicAdd(ctl + C_LIVE, (uint32_t)live);
    }
}

// Removes every live vertex of remaining degree <= level into F.
__global__ void __launch_bounds__(kCoreBlock) k_core_scan(int32_t n, const int32_t *deg,
                                                          int32_t *core, int32_t level,
                                                          int32_t *F, uint32_t *cnt) {
    const int lane = lane_id();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v0 = (int64_t)blockIdx.x * blockDim.x; v0 < n; v0 += stride) {
        const int64_t v = v0 + threadIdx.x;
        const bool take = v < n && core[v] < 0 && deg[v] <= level;
        if (take) core[v] = level;
        const uint64_t mask = __ballot(take);
        if (!mask) continue;
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(cnt, (uint32_t)__popcll(mask));
        base = __shfl(base, 0);
        if (take) F[base + lanes_below(mask)] = (int32_t)v;
    }
}

// One sub-round: a wave per removed vertex lowers its live neighbours'
// degrees; those reaching `level` are removed into F2.
__global__ void __launch_bounds__(kCoreBlock) k_core_process(const int32_t *__restrict__ off,
                                                             const int32_t *__restrict__ adj,
                                                             int32_t *deg, int32_t *core,
                                                             int32_t level, const int32_t *F,
                                                             int32_t cnt, int32_t *F2,
                                                             uint32_t *cnt2) {
    const int lane = lane_id();
    const int64_t nwaves = (int64_t)gridDim.x * kCoreWaves;
    for (int64_t i = (int64_t)blockIdx.x * kCoreWaves + threadIdx.x / kWave; i < cnt;
         i += nwaves) {
        const int32_t v = F[i];
        const int32_t e = off[v + 1];
        for (int32_t j0 = off[v]; j0 < e; j0 += kWave) {
            const int32_t j = j0 + lane;
            bool app = false;
            int32_t u = 0;
            if (j < e) {
                u = adj[j];
                if (core[u] < 0) {
                    const int32_t old = atomicSub(deg + u, 1);
                    if (old == level + 1) {
                        core[u] = level;
                        app = true;
                    }
                }
            }
            const uint64_t mask = __ballot(app);
            if (!mask) continue;
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(cnt2, (uint32_t)__popcll(mask));
            base = __shfl(base, 0);
            if (app) F2[base + lanes_below(mask)] = u;
        }
    }
}

__device__ __forceinline__ int32_t key_of(const int32_t *__restrict__ off,
                                          const int32_t *__restrict__ core, int32_t v) {
    return core ? core[v] : off[v + 1] - off[v];
}

// Out-degree of every row under the key order (a wave per row).
__global__ void __launch_bounds__(kCoreBlock) k_core_key(const int32_t *__restrict__ off,
                                                         const int32_t *__restrict__ core,
                                                         int32_t n, int32_t S, int32_t *key) {
    const int32_t cap = (int32_t)((1u << S) - 1u);
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        key[v] = (core[v] << S) | min(off[v + 1] - off[v], cap);
}

__global__ void __launch_bounds__(kCoreBlock) k_key_count(const int32_t *__restrict__ off,
                                                          const int32_t *__restrict__ adj,
                                                          int32_t n,
                                                          const int32_t *__restrict__ core,
                                                          int32_t *outcnt) {
    const int lane = lane_id();
    const int64_t nwaves = (int64_t)gridDim.x * kCoreWaves;
    for (int64_t r = (int64_t)blockIdx.x * kCoreWaves + threadIdx.x / kWave; r < n; r += nwaves) {
        const int32_t u = (int32_t)r, ku = key_of(off, core, u), e = off[u + 1];
        int32_t c = 0;
        for (int32_t j = off[u] + lane; j < e; j += kWave) {
            const int32_t v = adj[j];
            c += rank_less(ku, u, key_of(off, core, v), v) ? 1 : 0;
        }
        c = wave_sum(c);
        if (lane == 0) outcnt[u] = c;
    }
}

__global__ void __launch_bounds__(kCoreBlock) k_key_fill(const int32_t *__restrict__ off,
                                                         const int32_t *__restrict__ adj,
                                                         int32_t n,
                                                         const int32_t *__restrict__ core,
                                                         const int32_t *__restrict__ dag_off,
                                                         int32_t *dag_adj, int32_t *dag_src,
                                                         uint32_t *ctl) {
    const int lane = lane_id();
    const int64_t nwaves = (int64_t)gridDim.x * kCoreWaves;
    int32_t maxo = 0;
    for (int64_t r = (int64_t)blockIdx.x * kCoreWaves + threadIdx.x / kWave; r < n; r += nwaves) {
        const int32_t u = (int32_t)r, ku = key_of(off, core, u), e = off[u + 1];
        int32_t base = dag_off[u];
        for (int32_t j0 = off[u]; j0 < e; j0 += kWave) {
            const int32_t j = j0 + lane;
            int32_t v = 0;
            bool keep = false;
            if (j < e) {
                v = adj[j];
                keep = rank_less(ku, u, key_of(off, core, v), v);
            }
            const uint64_t mask = __ballot(keep);
            if (keep) {
                const int32_t p = base + lanes_below(mask);
                dag_adj[p] = v;
                dag_src[p] = u;
            }
            base += __popcll(mask);
        }
        maxo = max(maxo, base - dag_off[u]);
    }
    maxo = wave_max(maxo);
    if (lane == 0 && maxo > 0) atomicMax(ctl + C_MAX_OUT, (uint32_t)maxo);
}

struct CoreWs {
    int32_t *deg, *core, *F, *F2, *outcnt;
    int64_t *scan_tmp;
    uint32_t *ctl;
};

CoreWs core_layout(int32_t n, void *base, uint64_t *bytes) {
    Carve c(base, ~0ull);
    const uint64_t n1 = (uint64_t)n + 1;
    CoreWs W;
    W.deg = c.take<int32_t>(n1);
    W.core = c.take<int32_t>(n1);
    W.F = c.take<int32_t>(n1);
    W.F2 = c.take<int32_t>(n1);
    W.outcnt = c.take<int32_t>(n1);
    W.scan_tmp = c.take<int64_t>(scan_tmp_words(n1));
    W.ctl = c.take<uint32_t>(C_WORDS);
    if (bytes) *bytes = c.used;
    return W;
}

unsigned vgrid(int64_t items) {
    return (unsigned)std::max<int64_t>(
        1, std::min<int64_t>((items + kCoreBlock - 1) / kCoreBlock, (int64_t)cu_count() * 16));
}

unsigned wgrid(int64_t rows) {
    return (unsigned)std::max<int64_t>(
        1, std::min<int64_t>((rows + kCoreWaves - 1) / kCoreWaves, (int64_t)cu_count() * 16));
}

gpm_status read_u32(const uint32_t *d, uint32_t *h, int count, hipStream_t st) {
    GPM_HIP(hipMemcpyAsync(h, d, sizeof(uint32_t) * count, hipMemcpyDeviceToHost, st));
    GPM_HIP(hipStreamSynchronize(st));
    return GPM_OK;
}

}  // namespace

uint64_t orient_scratch_bytes(const gpm_graph *g) {
    uint64_t b = 0;
    core_layout(g->n, nullptr, &b);
    return b;
}

static gpm_status core_numbers_run(const gpm_graph *g, const CoreWs &W, hipStream_t st,
                                   int32_t *max_core) {
    const int32_t n = g->n;
    hipLaunchKernelGGL(k_core_init, dim3(vgrid(n)), dim3(kCoreBlock), 0, st, g->off, n, W.deg,
                       W.core);
    GPM_LAUNCH_CHECK("k_core_init");
    int32_t level = 0;
    *max_core = 0;
    for (;;) {
        GPM_HIP(fill_u32(W.ctl + C_MIN_DEG, 0xffffffffu, 1, st));
        GPM_HIP(fill_u32(W.ctl + C_LIVE, 0, 3, st));
        hipLaunchKernelGGL(k_core_stats, dim3(vgrid(n)), dim3(kCoreBlock), 0, st, n, W.deg,
                           W.core, W.ctl);
        GPM_LAUNCH_CHECK("k_core_stats");
        uint32_t h[2];
        gpm_status rc = read_u32(W.ctl, h, 2, st);
        if (rc) return rc;
        if (h[C_LIVE] == 0) break;
        level = std::max(level, (int32_t)h[C_MIN_DEG]);
        *max_core = level;
        hipLaunchKernelGGL(k_core_scan, dim3(vgrid(n)), dim3(kCoreBlock), 0, st, n, W.deg, W.core,
                           level, W.F, W.ctl + C_CNT0);
        GPM_LAUNCH_CHECK("k_core_scan");
        uint32_t cnt = 0;
        rc = read_u32(W.ctl + C_CNT0, &cnt, 1, st);
        if (rc) return rc;
        int32_t *cur = W.F, *nxt = W.F2;
        int slot = C_CNT0;
        while (cnt > 0) {
            const int nslot = slot == C_CNT0 ? C_CNT1 : C_CNT0;
            GPM_HIP(fill_u32(W.ctl + nslot, 0, 1, st));
            hipLaunchKernelGGL(k_core_process, dim3(wgrid(cnt)), dim3(kCoreBlock), 0, st, g->off,
                               g->adj, W.deg, W.core, level, cur, (int32_t)cnt, nxt,
                               W.ctl + nslot);
            GPM_LAUNCH_CHECK("k_core_process");
            rc = read_u32(W.ctl + nslot, &cnt, 1, st);
            if (rc) return rc;
            std::swap(cur, nxt);
            slot = nslot;
        }
        level++;
    }
    return GPM_OK;
}

gpm_status graph_orient(gpm_graph *g, int32_t order, void *scratch, uint64_t scratch_bytes,
                        int32_t *d_core, hipStream_t st) {
    uint64_t need = 0;
    CoreWs W = core_layout(g->n, scratch, &need);
    if (need > scratch_bytes) return fail(GPM_OUT_OF_MEMORY, "scratch smaller than required");
    const int32_t n = g->n;
    Span sp(order == GPM_ORIENT_CORE ? "graph_orient_core" : "graph_orient_degree", st);
    GPM_HIP(fill_u32(W.ctl, 0, C_WORDS, st));
    const int32_t *key = nullptr;
    if (order == GPM_ORIENT_CORE || d_core) {
        int32_t max_core = 0;
        gpm_status rc = core_numbers_run(g, W, st, &max_core);
        if (rc) return rc;
        if (d_core)
            GPM_HIP(hipMemcpyAsync(d_core, W.core, sizeof(int32_t) * (size_t)n,
                                   hipMemcpyDeviceToDevice, st));
        if (order == GPM_ORIENT_CORE) {
            int bits = 0;
            while (bits < 31 && (max_core >> bits) != 0) bits++;
            // the local-graph kernels order each root's out-neighbours by the
            // same key, so it is kept with the graph
            hipLaunchKernelGGL(k_core_key, dim3(vgrid(n)), dim3(kCoreBlock), 0, st, g->off,
                               W.core, n, 31 - bits, g->okey);
            GPM_LAUNCH_CHECK("k_core_key");
            key = g->okey;
        }
    }
    hipLaunchKernelGGL(k_key_count, dim3(wgrid(n)), dim3(kCoreBlock), 0, st, g->off, g->adj, n,
                       key, W.outcnt);
    GPM_LAUNCH_CHECK("k_key_count");
    GPM_HIP(exclusive_scan_i32(W.outcnt, g->dag_off, (uint64_t)n, W.scan_tmp, st));
    GPM_HIP(fill_u32(W.ctl + C_MAX_OUT, 0, 1, st));
    hipLaunchKernelGGL(k_key_fill, dim3(wgrid(n)), dim3(kCoreBlock), 0, st, g->off, g->adj, n,
                       key, g->dag_off, g->dag_adj, g->dag_src, W.ctl);
    GPM_LAUNCH_CHECK("k_key_fill");
    if (!key) GPM_HIP(degree_key(g->off, n, g->okey, st));
    uint32_t maxo = 0;
    gpm_status rc = read_u32(W.ctl + C_MAX_OUT, &maxo, 1, st);
    if (rc) return rc;
    g->max_out_degree = (int32_t)maxo;
    return GPM_OK;
}

}  // namespace gpm
