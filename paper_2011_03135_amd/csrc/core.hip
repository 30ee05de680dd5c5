// Core numbers and the core-value orientation (Appendix B.2 names two
// orientations for cliques: by degree and by core value).
//
// Core numbers by level-synchronous peeling.  For level L = 0, 1, ...: every
// vertex not yet removed whose remaining degree is at most L is removed with
// core number L (a scan), and removing a vertex lowers its live neighbours'
// remaining degrees (atomic decrements); a neighbour whose degree falls from
// L + 1 to L is removed at the same level, in the next sub-round.  Each
// vertex is removed once, when the decrement that takes it to L is the one
// that sees L + 1, so the frontier lists never repeat a vertex.  Levels with
// nothing to remove are skipped by taking the smallest remaining degree.
//
// Scans and sub-rounds are steps of one kernel, k_core_step, queued back to
// back.  A step reads the peeling state (level, scan or sub-round, its
// input frontier's size) that the previous step left, does its share, and
// the last workgroup to finish (a count of finished workgroups) turns the
// step's counters into the next state; the kernel boundary orders the steps,
// so no workgroup ever waits for another.  The host queues steps in batches
// and reads the state once per batch; steps queued past the end do nothing.
// Scans walk a list of the vertices still live at the previous scan (all of
// them at the first) and write the ones they keep to a second list, so a
// scan costs the live vertices rather than n.
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

// ctl words: the peeling state (level; mode; input frontier size and which
// frontier buffer holds it; live-list size and buffer; first scan; largest
// core so far), the finished-workgroup count, the step's counters (output
// size, smallest kept degree, vertices kept) and the orientation's largest
// out-degree
enum { S_LEVEL = 0, S_MODE = 1, S_CIN = 2, S_FBUF = 3, S_LIVE = 4, S_LBUF = 5, S_FIRST = 6,
       S_MAXCORE = 7, S_DONE = 8, K_CNT = 9, K_MIN = 10, K_KEPT = 11, C_MAX_OUT = 12,
       C_WORDS = 16 };
enum { M_SCAN = 0, M_PROCESS = 1, M_END = 2 };

__global__ void __launch_bounds__(kCoreBlock) k_core_init(const int32_t *__restrict__ off,
                                                          int32_t n, int32_t *deg,
                                                          int32_t *core) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        deg[v] = off[v + 1] - off[v];
        core[v] = -1;
    }
}

// One step of the peeling (see above).  F0/F1: frontier buffers (scans
// write F0, sub-rounds alternate); L0/L1: live lists.
__global__ void __launch_bounds__(kCoreBlock) k_core_step(const int32_t *__restrict__ off,
                                                          const int32_t *__restrict__ adj,
                                                          int32_t n, int32_t *deg, int32_t *core,
                                                          int32_t *F0, int32_t *F1, int32_t *L0,
                                                          int32_t *L1, uint32_t *ctl) {
    __shared__ int32_t wmin[kCoreWaves];
    const uint32_t mode = ctl[S_MODE];
    if (mode == M_END) return;
    const int32_t level = (int32_t)ctl[S_LEVEL];
    const int lane = lane_id();
    if (mode == M_SCAN) {
        // live vertices of remaining degree <= level into F0, the others to
        // the other live list; the smallest degree kept, for skipping levels
        const bool first = ctl[S_FIRST] != 0;
        const int64_t live = first ? (int64_t)n : (int64_t)ctl[S_LIVE];
        const int32_t *lin = ctl[S_LBUF] ? L1 : L0;
        int32_t *lout = ctl[S_LBUF] ? L0 : L1;
        const int64_t stride = (int64_t)gridDim.x * blockDim.x;
        int32_t mn = INT_MAX;
        for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < live; i0 += stride) {
            const int64_t i = i0 + threadIdx.x;
            int32_t v = -1;
            if (i < live) v = first ? (int32_t)i : lin[i];
            const bool alive = v >= 0 && core[v] < 0;
            const int32_t d = alive ? deg[v] : INT_MAX;
            const bool take = alive && d <= level;
            const bool keep = alive && !take;
            if (take) core[v] = level;
            else mn = min(mn, d);
            const uint64_t tmask = __ballot(take), kmask = __ballot(keep);
            if (tmask) {
                uint32_t base = 0;
                if (lane == 0) base = atomicAdd(ctl + K_CNT, (uint32_t)__popcll(tmask));
                base = __shfl(base, 0);
                if (take) F0[base + lanes_below(tmask)] = v;
            }
            if (kmask) {
                uint32_t base = 0;
                if (lane == 0) base = atomicAdd(ctl + K_KEPT, (uint32_t)__popcll(kmask));
                base = __shfl(base, 0);
                if (keep) lout[base + lanes_below(kmask)] = v;
            }
        }
        // one atomic per workgroup: a per-wave atomic on one word
        // serialises thousands of waves
        mn = -wave_max(-mn);
        if (lane == 0) wmin[threadIdx.x / kWave] = mn;
        __syncthreads();
        if (threadIdx.x == 0) {
            int32_t b = wmin[0];
            for (int w = 1; w < kCoreWaves; w++) b = min(b, wmin[w]);
            if (b != INT_MAX) atomicMin(ctl + K_MIN, (uint32_t)b);
        }
    } else {
        // one sub-round: a wave per removed vertex lowers its live
        // neighbours' degrees; those reaching the level are removed
        const int32_t *fin = ctl[S_FBUF] ? F1 : F0;
        int32_t *fout = ctl[S_FBUF] ? F0 : F1;
        const int64_t cin = (int64_t)ctl[S_CIN];
        const int64_t nwaves = (int64_t)gridDim.x * kCoreWaves;
        for (int64_t i = (int64_t)blockIdx.x * kCoreWaves + threadIdx.x / kWave; i < cin;
             i += nwaves) {
            const int32_t v = fin[i];
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
                if (lane == 0) base = atomicAdd(ctl + K_CNT, (uint32_t)__popcll(mask));
                base = __shfl(base, 0);
                if (app) fout[base + lanes_below(mask)] = u;
            }
        }
    }
    // the last workgroup to finish sets the next state (every workgroup has
    // read the current one by then) and clears the step's counters.  Only
    // the counters cross workgroups inside the step, and they are device
    // atomics: each workgroup's counter updates are complete (the barrier
    // waits for its memory operations) before it counts itself finished,
    // and the last one reads them with atomic operations.  The frontier and
    // list entries reach the next step through the kernel boundary, so no
    // device-wide fence (a write-back of every L2) is needed here.
    __syncthreads();
    if (threadIdx.x != 0) return;
    __builtin_amdgcn_s_waitcnt(0);
    if (atomicAdd(ctl + S_DONE, 1u) != gridDim.x - 1) return;
    const uint32_t cnt = atomicAdd(ctl + K_CNT, 0u);
    const uint32_t kmin = atomicMin(ctl + K_MIN, 0xffffffffu);
    const uint32_t kept = atomicAdd(ctl + K_KEPT, 0u);
    if (mode == M_SCAN) {
        ctl[S_LIVE] = kept;
        ctl[S_LBUF] ^= 1u;
        ctl[S_FIRST] = 0u;
        if (cnt == 0) {
            if (kmin == 0xffffffffu) ctl[S_MODE] = M_END;   // nothing live
            else ctl[S_LEVEL] = (uint32_t)max(level + 1, (int32_t)kmin);
        } else {
            ctl[S_MAXCORE] = (uint32_t)level;
            ctl[S_MODE] = M_PROCESS;
            ctl[S_CIN] = cnt;
            ctl[S_FBUF] = 0u;
        }
    } else if (cnt == 0) {
        ctl[S_LEVEL] = (uint32_t)(level + 1);
        ctl[S_MODE] = M_SCAN;
    } else {
        ctl[S_CIN] = cnt;
        ctl[S_FBUF] ^= 1u;
    }
    ctl[K_CNT] = 0u;
    ctl[K_MIN] = 0xffffffffu;
    ctl[K_KEPT] = 0u;
    ctl[S_DONE] = 0u;
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
    int32_t *deg, *core, *F, *F2, *L, *L2, *outcnt;
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
    W.L = c.take<int32_t>(n1);
    W.L2 = c.take<int32_t>(n1);
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
        if (hipHostMalloc(&q, sizeof(uint32_t) * C_WORDS, hipHostMallocDefault) == hipSuccess)
            p = static_cast<uint32_t *>(q);
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

// Steps queued per read of the state (RMAT-20 takes about 2,000 steps).
constexpr int kStepsPerTrip = 32;

static gpm_status core_numbers_run(const gpm_graph *g, const CoreWs &W, hipStream_t st,
                                   int32_t *max_core) {
    const int32_t n = g->n;
    hipLaunchKernelGGL(k_core_init, dim3(vgrid(n)), dim3(kCoreBlock), 0, st, g->off, n, W.deg,
                       W.core);
    GPM_LAUNCH_CHECK("k_core_init");
    GPM_HIP(fill_u32(W.ctl, 0, C_WORDS, st));
    GPM_HIP(fill_u32(W.ctl + K_MIN, 0xffffffffu, 1, st));
    GPM_HIP(fill_u32(W.ctl + S_FIRST, 1u, 1, st));
    // one workgroup per CU: most steps are small and a step's cost is
    // mostly its launch and completion, which grow with the grid (RMAT-20:
    // 17.8 ms at 256 workgroups, 18.1 at 128, 20.4 at 512, 25.3 at 1024)
    const unsigned pgrid = (unsigned)std::max(1, cu_count());
    // a level with removals takes a scan that removes a vertex, sub-rounds
    // that each remove one more but the last, and at most one skipping scan
    // before it; so at most 4n + 1 steps
    const int64_t max_trips = (4 * (int64_t)n + 1) / kStepsPerTrip + 2;
    uint32_t h[C_WORDS];
    Span sp("k_core_step", st);
    for (int64_t trip = 0;; trip++) {
        if (trip > max_trips) return fail(GPM_DEVICE_ERROR, "core peeling did not finish");
        for (int r = 0; r < kStepsPerTrip; r++)
            hipLaunchKernelGGL(k_core_step, dim3(pgrid), dim3(kCoreBlock), 0, st, g->off, g->adj,
                               n, W.deg, W.core, W.F, W.F2, W.L, W.L2, W.ctl);
        GPM_LAUNCH_CHECK("k_core_step");
        gpm_status rc = read_u32(W.ctl, h, C_WORDS, st);
        if (rc) return rc;
        if (h[S_MODE] == M_END) break;
    }
    *max_core = (int32_t)h[S_MAXCORE];
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
