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
// smallest remaining degree.  The host drives the levels; sub-rounds are
// queued two at a time between reads of the counters.
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
#include <mutex>

#include "gpm_internal.h"

namespace gpm {

namespace {

constexpr int kCoreBlock = 256;
constexpr int kCoreWaves = kCoreBlock / kWave;

// ctl words: smallest degree left, vertices removed so far, the scan's and
// the sub-rounds' frontier sizes (two alternating slots)
enum { C_MIN_DEG = 0, C_REMOVED = 1, C_SCAN = 2, C_CNT0 = 3, C_CNT1 = 4, C_MAX_OUT = 5,
       C_WORDS = 8 };

__global__ void __launch_bounds__(kCoreBlock) k_core_init(const int32_t *__restrict__ off,
                                                          int32_t n, int32_t *deg,
                                                          int32_t *core) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        deg[v] = off[v + 1] - off[v];
        core[v] = -1;
    }
}

// Removes every live vertex of remaining degree <= level into F (count in
// ctl[C_SCAN]) and leaves the smallest degree among the live vertices it
// keeps in ctl[C_MIN_DEG], for skipping empty levels.
__global__ void __launch_bounds__(kCoreBlock) k_core_scan(int32_t n, const int32_t *deg,
                                                          int32_t *core, int32_t level,
                                                          int32_t *F, uint32_t *ctl) {
    const int lane = lane_id();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int32_t mn = INT_MAX;
    for (int64_t v0 = (int64_t)blockIdx.x * blockDim.x; v0 < n; v0 += stride) {
        const int64_t v = v0 + threadIdx.x;
        const bool live = v < n && core[v] < 0;
        const int32_t d = live ? deg[v] : INT_MAX;
        const bool take = live && d <= level;
        if (take) core[v] = level;
        else mn = min(mn, d);
        const uint64_t mask = __ballot(take);
        if (!mask) continue;
        uint32_t base = 0;
        if (lane == 0) {
            base = atomicAdd(ctl + C_SCAN, (uint32_t)__popcll(mask));
            atomicAdd(ctl + C_REMOVED, (uint32_t)__popcll(mask));
        }
        base = __shfl(base, 0);
        if (take) F[base + lanes_below(mask)] = (int32_t)v;
    }
    // one atomic per workgroup: a per-wave atomic on one word serialises
    // thousands of waves
    __shared__ int32_t wmin[kCoreWaves];
    mn = -wave_max(-mn);
    if (lane == 0) wmin[threadIdx.x / kWave] = mn;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t b = wmin[0];
        for (int w = 1; w < kCoreWaves; w++) b = min(b, wmin[w]);
        if (b != INT_MAX) atomicMin(ctl + C_MIN_DEG, (uint32_t)b);
    }
}

// One sub-round: a wave per removed vertex lowers its live neighbours'
// degrees; those reaching `level` are removed into F2.  The frontier's size
// is read on the device, so sub-rounds can be queued without a host trip.
__global__ void __launch_bounds__(kCoreBlock) k_core_process(const int32_t *__restrict__ off,
                                                             const int32_t *__restrict__ adj,
                                                             int32_t *deg, int32_t *core,
                                                             int32_t level, const int32_t *F,
                                                             const uint32_t *cnt_in, int32_t *F2,
                                                             uint32_t *cnt2, uint32_t *removed) {
    const int lane = lane_id();
    const int64_t nwaves = (int64_t)gridDim.x * kCoreWaves;
    const int64_t cnt = *cnt_in;
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
            if (lane == 0) {
                base = atomicAdd(cnt2, (uint32_t)__popcll(mask));
                atomicAdd(removed, (uint32_t)__popcll(mask));
            }
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

// A small pinned host buffer for the per-round counters (allocated once per
// process; pageable copies cost several times more per round trip).  It is
// shared by every thread, so read_u32 holds its mutex from the copy to the
// copy-out: concurrent orientations (other graphs, other streams, other
// threads) take turns at the buffer instead of reading each other's words.
std::mutex &pinned_mutex() {
    static std::mutex mu;
    return mu;
}

uint32_t *pinned_words_locked() {
    static uint32_t *p = nullptr;
    if (!p) {
        void *q = nullptr;
        if (hipHostMalloc(&q, 64, hipHostMallocDefault) == hipSuccess) p = static_cast<uint32_t *>(q);
    }
    return p;
}

gpm_status read_u32(const uint32_t *d, uint32_t *h, int count, hipStream_t st) {
    std::lock_guard<std::mutex> lock(pinned_mutex());
    uint32_t *pin = pinned_words_locked();
    GPM_HIP(hipMemcpyAsync(pin ? pin : h, d, sizeof(uint32_t) * count, hipMemcpyDeviceToHost,
                           st));
    GPM_HIP(hipStreamSynchronize(st));
    if (pin)
        for (int i = 0; i < count; i++) h[i] = pin[i];
    return GPM_OK;
}

}  // namespace

uint64_t orient_scratch_bytes(const gpm_graph *g) {
    uint64_t b = 0;
    core_layout(g->n, nullptr, &b);
    return b;
}

// Sub-rounds queued per host round trip: most levels need one to three.
constexpr int kRoundsPerTrip = 2;

static gpm_status core_numbers_run(const gpm_graph *g, const CoreWs &W, hipStream_t st,
                                   int32_t *max_core) {
    const int32_t n = g->n;
    hipLaunchKernelGGL(k_core_init, dim3(vgrid(n)), dim3(kCoreBlock), 0, st, g->off, n, W.deg,
                       W.core);
    GPM_LAUNCH_CHECK("k_core_init");
    GPM_HIP(fill_u32(W.ctl, 0, C_WORDS, st));
    const unsigned pgrid = (unsigned)std::max(1, cu_count() * 4);
    int32_t level = 0;
    *max_core = 0;
    uint32_t removed = 0;
    while (removed < (uint32_t)n) {
        GPM_HIP(fill_u32(W.ctl + C_MIN_DEG, 0xffffffffu, 1, st));
        GPM_HIP(fill_u32(W.ctl + C_SCAN, 0, 1, st));
        hipLaunchKernelGGL(k_core_scan, dim3(pgrid), dim3(kCoreBlock), 0, st, n, W.deg, W.core,
                           level, W.F, W.ctl);
        GPM_LAUNCH_CHECK("k_core_scan");
        // sub-rounds: the scan's frontier (F, count in C_SCAN), then
        // alternating F2 / F with counts in C_CNT0 / C_CNT1
        const uint32_t *cin = W.ctl + C_SCAN;
        int32_t *cur = W.F, *nxt = W.F2;
        int slot = C_CNT0;
        uint32_t h[8];
        bool first = true;
        for (;;) {
            for (int r = 0; r < kRoundsPerTrip; r++) {
                GPM_HIP(fill_u32(W.ctl + slot, 0, 1, st));
                hipLaunchKernelGGL(k_core_process, dim3(pgrid), dim3(kCoreBlock), 0, st, g->off,
                                   g->adj, W.deg, W.core, level, cur, cin, nxt, W.ctl + slot,
                                   W.ctl + C_REMOVED);
                GPM_LAUNCH_CHECK("k_core_process");
                cin = W.ctl + slot;
                slot = slot == C_CNT0 ? C_CNT1 : C_CNT0;
                std::swap(cur, nxt);
            }
            gpm_status rc = read_u32(W.ctl, h, C_WORDS, st);
            if (rc) return rc;
            if (first && h[C_SCAN] == 0) break;   // nothing at this level
            first = false;
            if (h[cin - W.ctl] == 0) break;   // the last sub-round removed nothing
        }
        removed = h[C_REMOVED];
        if (h[C_SCAN] == 0) {
            // skip to the smallest remaining degree
            if (h[C_MIN_DEG] == 0xffffffffu) break;
            level = std::max(level + 1, (int32_t)h[C_MIN_DEG]);
            continue;
        }
        *max_core = level;
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
