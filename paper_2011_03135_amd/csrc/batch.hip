// Batched 3- and 4-motif counting of many small graphs in one pass.
//
// The G graphs are one union graph g whose graph i owns vertices
// voff[i] .. voff[i+1]-1.  Teams of threads (one workgroup per graph at a
// time, graphs popped from an atomic cursor) compute every step of the motif
// path for their graph entirely on chip: the graph's offsets are staged in
// LDS, its adjacency becomes bit rows in LDS (row v = neighbours of v,
// ceil(n/64) words), and
//   degrees             d_v = |A_v|
//   per-edge triangles  T_uv = |A_u & A_v|               (Section 5)
//   local-count sums    the four per-edge sums of the motif path
//   4-cliques           sum over triangles u < v < w of |A_u & A_v & A_w & above(w)|
//   4-cycles            sum over x, z < x of C(|A_x & A_z & below(x)|, 2)
//                       (each cycle once, from its largest vertex x and the
//                       opposite vertex z; the middles lie below x)
// are combined into the induced counts with the same exact identities as the
// single-graph path, and written to the graph's row of the output.
//
// Scheduling.  A counting sort orders the graphs by vertex count, largest
// first (longest job first, so the last teams to finish hold the smallest
// graphs).  The sorted order is cut into tiers by row width (graphs of at
// most 64, 128, 256 and 1024 vertices); each tier is one persistent launch
// whose LDS is sized for its widest graph, so narrow graphs are not held to
// the occupancy of wide ones.  Team width, the tiers used below 256 vertices
// and the teams per compute unit are run-time choices (gpm_batch_config);
// gpm_batch_autotune times the candidates on the caller's batch.
#include "gpm_internal.h"

#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

namespace gpm {

namespace {

typedef unsigned __int128 u128;

constexpr int kMaxN = GPM_BATCH_MAX_VERTICES;
constexpr int kLargeNT = 256;
constexpr int kHist = kMaxN + 1;   // vertex counts 0 .. kMaxN

enum BatchFlags : unsigned long long {
    B_DIVISION = 1,       // an exact division of the combining identities failed
    B_TOO_LARGE = 64,     // graph has more than GPM_BATCH_MAX_VERTICES vertices
    B_BAD_RANGE = 128,    // voff not ascending or beyond n
    B_CROSS_EDGE = 256,   // an edge leaves the graph's vertex range
};

// Workspace (int32 words): hist[kHist], gt[kHist + 1] (gt[b] = number of
// sortable graphs with more than b vertices, b <= kMaxN; gt[kHist] = number
// of sortable graphs), cur[kHist] (scatter cursors), tier cursors[8],
// order[G] (sortable graphs by vertex count, descending).
struct BatchWs {
    int32_t *hist, *gt, *cur;
    uint32_t *tcur;
    int32_t *order;
};

constexpr int64_t kWsHead = 3 * (int64_t)kHist + 1 + 8;

BatchWs batch_ws(void *ws) {
    int32_t *w = static_cast<int32_t *>(ws);
    BatchWs b;
    b.hist = w;
    b.gt = w + kHist;
    b.cur = w + 2 * kHist + 1;
    b.tcur = reinterpret_cast<uint32_t *>(w + 3 * kHist + 1);
    b.order = w + kWsHead;
    return b;
}

__device__ __forceinline__ uint64_t below_mask(int32_t x, int32_t w) {
    // bits < x within word w
    const int32_t lo = w * 64;
    if (x <= lo) return 0ull;
    if (x >= lo + 64) return ~0ull;
    return (1ull << (x - lo)) - 1ull;
}

// Exact combination (one thread); flags |= B_DIVISION on a failed check.
__device__ void combine(int32_t k, u128 wedge, u128 tri, u128 k4, u128 s1, u128 s2, u128 s3,
                        u128 s4, u128 nc4, unsigned long long flags, unsigned long long *out) {
    if (k == 3) {
        unsigned long long bad = flags;
        if (wedge < 3 * tri) bad |= B_DIVISION;
        out[0] = (unsigned long long)(wedge - 3 * tri);
        out[1] = (unsigned long long)tri;
        out[2] = bad;
        return;
    }
    unsigned long long bad = flags;
    u128 dia = 0, paw = 0, c4 = 0, p4 = 0, claw = 0;
    if (s1 < 6 * k4) bad |= B_DIVISION; else dia = s1 - 6 * k4;
    if (s2 < 4 * dia || ((s2 - 4 * dia) & 1)) bad |= B_DIVISION; else paw = (s2 - 4 * dia) / 2;
    if (nc4 < dia + 3 * k4) bad |= B_DIVISION; else c4 = nc4 - dia - 3 * k4;
    if (s3 < 4 * c4) bad |= B_DIVISION; else p4 = s3 - 4 * c4;
    if (s4 < paw || (s4 - paw) % 3) bad |= B_DIVISION; else claw = (s4 - paw) / 3;
    out[0] = (unsigned long long)claw;
    out[1] = (unsigned long long)p4;
    out[2] = (unsigned long long)c4;
    out[3] = (unsigned long long)paw;
    out[4] = (unsigned long long)dia;
    out[5] = (unsigned long long)k4;
    out[6] = bad;
}

// ------------------------------------------------------------ ordering ---

// Per graph: flags graphs no tier can take (their rows are written here) and
// histograms the vertex counts of the others.
__global__ void k_batch_hist(const int32_t *__restrict__ voff, int32_t G, int32_t n, int32_t k,
                             int32_t *hist, unsigned long long *counts) {
    const int width = k == 3 ? 3 : 7;
    for (int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gi < G;
         gi += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v0 = voff[gi], v1 = voff[gi + 1];
        unsigned long long bad = 0;
        if (v0 < 0 || v1 < v0 || v1 > n) bad = B_BAD_RANGE;
        else if (v1 - v0 > kMaxN) bad = B_TOO_LARGE;
        if (bad) {
            unsigned long long *out = counts + gi * width;
            for (int q = 0; q < width - 1; q++) out[q] = 0;
            out[width - 1] = bad;
        } else {
            atomicAdd(&hist[v1 - v0], 1);
        }
    }
}

// One wave: gt[b] = sum of hist[b'] over b' > b; cur = gt (scatter cursors);
// gt[kHist] = total.  Lane l owns the reversed indices r = l*kPer ..
// (l+1)*kPer - 1 (b = kMaxN - r).
__global__ void __launch_bounds__(kWave) k_batch_scan(const int32_t *hist, int32_t *gt,
                                                      int32_t *cur) {
    constexpr int kPer = (kHist + kWave - 1) / kWave;
    const int l = lane_id();
    int32_t loc[kPer];
    int32_t s = 0;
#pragma unroll
    for (int i = 0; i < kPer; i++) {
        const int r = l * kPer + i;
        loc[i] = r < kHist ? hist[kMaxN - r] : 0;
        s += loc[i];
    }
    int32_t before = wave_incl_scan(s) - s;
#pragma unroll
    for (int i = 0; i < kPer; i++) {
        const int r = l * kPer + i;
        if (r < kHist) {
            gt[kMaxN - r] = before;   // graphs with more than b vertices
            cur[kMaxN - r] = before;
        }
        before += loc[i];
    }
    if (l == kWave - 1) gt[kHist] = before;
}

__global__ void k_batch_scatter(const int32_t *__restrict__ voff, int32_t G, int32_t n,
                                int32_t *cur, int32_t *order) {
    for (int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gi < G;
         gi += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v0 = voff[gi], v1 = voff[gi + 1];
        if (v0 < 0 || v1 < v0 || v1 > n || v1 - v0 > kMaxN) continue;
        order[atomicAdd(&cur[v1 - v0], 1)] = (int32_t)gi;
    }
}

// ------------------------------------------------------------- mining ---

template <int NMAX, int NT>
struct BatchLds {
    static constexpr int W = NMAX / 64;
    uint64_t rows[NMAX * W];
    int32_t deg[NMAX];
    int32_t off[NMAX + 1];   // arc offsets relative to the graph's first arc
    unsigned long long part[NT / kWave][8];
    unsigned long long flags;
    uint32_t task;
};

template <int NMAX, int NT>
__device__ unsigned long long block_sum(BatchLds<NMAX, NT> &sh, unsigned long long x, int slot) {
    x = wave_sum(x);
    if (lane_id() == 0) sh.part[threadIdx.x / kWave][slot] = x;
    __syncthreads();
    unsigned long long s = 0;
    for (int q = 0; q < NT / kWave; q++) s += sh.part[q][slot];
    return s;
}

// Vertex owning relative arc r: the last i in [0, ng) with off[i] <= r.
__device__ __forceinline__ int32_t arc_owner(const int32_t *off, int32_t ng, int32_t r) {
    int32_t lo = 0, hi = ng;
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (off[mid] <= r) lo = mid; else hi = mid;
    }
    return lo;
}

// Mines the graphs at sorted positions gt[hi_b] .. gt[lo_b]-1, i.e. those
// with lo_b < n_g <= hi_b (lo_b = -1: through the end of the order).
template <int NMAX, int NT>
__global__ void __launch_bounds__(NT) k_batch(const int32_t *__restrict__ off,
                                              const int32_t *__restrict__ adj,
                                              const int32_t *__restrict__ voff,
                                              const int32_t *__restrict__ order,
                                              const int32_t *__restrict__ gt, int32_t lo_b,
                                              int32_t k, uint32_t *cursor,
                                              unsigned long long *counts) {
    constexpr int W = NMAX / 64;
    __shared__ BatchLds<NMAX, NT> sh;
    const int tid = threadIdx.x;
    const int width = k == 3 ? 3 : 7;
    const int32_t p_begin = gt[NMAX];
    const int32_t p_end = gt[lo_b < 0 ? kHist : lo_b];
    for (;;) {
        if (tid == 0) sh.task = atomicAdd(cursor, 1u);
        __syncthreads();
        const int32_t p = p_begin + (int32_t)sh.task;
        __syncthreads();
        if (p >= p_end) break;
        const int32_t gi = order[p];
        const int32_t v0 = voff[gi], ng = voff[gi + 1] - v0;
        unsigned long long *out = counts + (int64_t)gi * width;
        const int32_t Wg = (ng + 63) >> 6;
        const int32_t a0 = off[v0];
        for (int32_t i = tid; i < ng * W; i += NT) sh.rows[i] = 0ull;
        for (int32_t i = tid; i <= ng; i += NT) sh.off[i] = off[v0 + i] - a0;
        if (tid == 0) sh.flags = 0;
        __syncthreads();
        const int32_t na = sh.off[ng];
        for (int32_t r = tid; r < na; r += NT) {
            const int32_t w = adj[a0 + r] - v0;
            if (w < 0 || w >= ng) {
                atomicOr(&sh.flags, (unsigned long long)B_CROSS_EDGE);
                continue;
            }
            const int32_t u = arc_owner(sh.off, ng, r);
            atomicOr((unsigned long long *)&sh.rows[u * W + (w >> 6)], 1ull << (w & 63));
        }
        __syncthreads();
        unsigned long long wedge = 0;
        for (int32_t v = tid; v < ng; v += NT) {
            int32_t d = 0;
            for (int32_t q = 0; q < Wg; q++) d += __popcll(sh.rows[v * W + q]);
            sh.deg[v] = d;
            wedge += (unsigned long long)d * (d - (d > 0)) / 2;
        }
        __syncthreads();
        unsigned long long tri3 = 0, s1 = 0, s2 = 0, s3 = 0, s4 = 0, k4 = 0, c4 = 0;
        // edges u < v, one arc per thread
        for (int32_t r = tid; r < na; r += NT) {
            const int32_t v = adj[a0 + r] - v0;
            if (v < 0 || v >= ng) continue;
            const int32_t u = arc_owner(sh.off, ng, r);
            if (!(u < v)) continue;
            const uint64_t *ru = sh.rows + u * W, *rv = sh.rows + v * W;
            uint64_t t = 0;
            for (int32_t q = 0; q < Wg; q++) t += __popcll(ru[q] & rv[q]);
            tri3 += t;
            if (k == 4) {
                const uint64_t su = sh.deg[u] - t - 1, sv = sh.deg[v] - t - 1;
                s1 += t * (t - (t > 0)) / 2;
                s2 += t * (su + sv);
                s3 += su * sv;
                s4 += su * (su - (su > 0)) / 2 + sv * (sv - (sv > 0)) / 2;
                // 4-cliques u < v < x < y
                for (int32_t q = v >> 6; q < Wg; q++) {
                    uint64_t c = ru[q] & rv[q] & ~below_mask(v + 1, q);
                    while (c) {
                        const int32_t x = q * 64 + __builtin_ctzll(c);
                        c &= c - 1;
                        const uint64_t *rx = sh.rows + x * W;
                        for (int32_t r2 = x >> 6; r2 < Wg; r2++)
                            k4 += __popcll(ru[r2] & rv[r2] & rx[r2] & ~below_mask(x + 1, r2));
                    }
                }
            }
        }
        if (k == 4) {
            // 4-cycles from their largest vertex x and opposite vertex z < x;
            // pair p = x(x-1)/2 + z, p < 2^19, so the float root is within 1
            const int32_t npairs = ng * (ng - 1) / 2;
            for (int32_t p2 = tid; p2 < npairs; p2 += NT) {
                int32_t x = (int32_t)((1.0f + sqrtf(1.0f + 8.0f * (float)p2)) * 0.5f);
                while (x * (x - 1) / 2 > p2) x--;
                while ((x + 1) * x / 2 <= p2) x++;
                const int32_t z = p2 - x * (x - 1) / 2;
                const uint64_t *rx = sh.rows + x * W, *rz = sh.rows + z * W;
                uint64_t c = 0;
                for (int32_t q = 0; q < Wg; q++) c += __popcll(rx[q] & rz[q] & below_mask(x, q));
                c4 += c * (c - (c > 0)) / 2;
            }
        }
        const unsigned long long W_ = block_sum(sh, wedge, 0);
        const unsigned long long T3 = block_sum(sh, tri3, 1);
        const unsigned long long S1 = block_sum(sh, s1, 2), S2 = block_sum(sh, s2, 3);
        const unsigned long long S3 = block_sum(sh, s3, 4), S4 = block_sum(sh, s4, 5);
        const unsigned long long K4 = block_sum(sh, k4, 6), C4 = block_sum(sh, c4, 7);
        if (tid == 0) {
            unsigned long long fl = sh.flags;
            if (T3 % 3) fl |= B_DIVISION;
            combine(k, W_, T3 / 3, K4, S1, S2, S3, S4, C4, fl, out);
        }
        __syncthreads();
    }
}

template <int NMAX, int NT>
void launch_tier(const gpm_graph *g, const int32_t *voff, const BatchWs &b, int32_t lo_b,
                 int32_t k, uint32_t *cursor, int blocks, unsigned long long *counts,
                 hipStream_t st) {
    hipLaunchKernelGGL((k_batch<NMAX, NT>), dim3((unsigned)blocks), dim3(NT), 0, st, g->off,
                       g->adj, voff, b.order, b.gt, lo_b, k, cursor, counts);
}

template <int NMAX>
void launch_small(int nt, const gpm_graph *g, const int32_t *voff, const BatchWs &b,
                  int32_t lo_b, int32_t k, uint32_t *cursor, int blocks,
                  unsigned long long *counts, hipStream_t st) {
    if (nt == 64) launch_tier<NMAX, 64>(g, voff, b, lo_b, k, cursor, blocks, counts, st);
    else if (nt == 128) launch_tier<NMAX, 128>(g, voff, b, lo_b, k, cursor, blocks, counts, st);
    else launch_tier<NMAX, 256>(g, voff, b, lo_b, k, cursor, blocks, counts, st);
}

}  // namespace

gpm_status batch_default_config(gpm_batch_config *c) {
    c->team_threads = 64;
    c->tiers = 3;
    c->blocks_per_cu = 16;
    c->reserved = 0;
    return GPM_OK;
}

gpm_status batch_check_config(const gpm_batch_config *c) {
    if (c->team_threads != 64 && c->team_threads != 128 && c->team_threads != 256)
        return fail(GPM_INVALID_ARGUMENT, "team_threads must be 64, 128 or 256");
    if (c->tiers < 1 || c->tiers > 3) return fail(GPM_INVALID_ARGUMENT, "tiers must be 1, 2 or 3");
    if (c->blocks_per_cu < 1 || c->blocks_per_cu > 32)
        return fail(GPM_INVALID_ARGUMENT, "blocks_per_cu must be in [1, 32]");
    return GPM_OK;
}

gpm_status batch_workspace_bytes(int32_t G, int32_t k, uint64_t *bytes) {
    (void)k;
    *bytes = ((uint64_t)(kWsHead + G) * 4 + 255) / 256 * 256;
    return GPM_OK;
}

gpm_status batch_run(const gpm_graph *g, const int32_t *d_voff, int32_t G, int32_t k,
                     const gpm_batch_config *cfg, void *ws, uint64_t ws_bytes,
                     unsigned long long *d_counts, hipStream_t st) {
    uint64_t need = 0;
    batch_workspace_bytes(G, k, &need);
    if (ws_bytes < need) return fail(GPM_OUT_OF_MEMORY, "workspace smaller than required");
    gpm_status rc = batch_check_config(cfg);
    if (rc) return rc;
    const BatchWs b = batch_ws(ws);
    const int cus = cu_count();
    const int eblocks = (int)std::min<int64_t>(((int64_t)G + 255) / 256, (int64_t)cus * 8);
    {
        Span sp("batch_order", st);
        GPM_HIP(fill_u32(b.hist, 0, kHist, st));
        GPM_HIP(fill_u32(b.tcur, 0, 8, st));
        hipLaunchKernelGGL(k_batch_hist, dim3((unsigned)eblocks), dim3(256), 0, st, d_voff, G,
                           g->n, k, b.hist, d_counts);
        hipLaunchKernelGGL(k_batch_scan, dim3(1), dim3(kWave), 0, st, b.hist, b.gt, b.cur);
        hipLaunchKernelGGL(k_batch_scatter, dim3((unsigned)eblocks), dim3(256), 0, st, d_voff,
                           G, g->n, b.cur, b.order);
    }
    GPM_LAUNCH_CHECK("batch_order");
    // tiers by row width, widest first; each takes (next narrower bound, own bound]
    const int nt = cfg->team_threads;
    const int small = (int)std::min<int64_t>(G, (int64_t)cus * cfg->blocks_per_cu);
    {
        Span sp("k_batch<1024>", st);
        launch_tier<kMaxN, kLargeNT>(g, d_voff, b, 256, k, b.tcur + 0,
                                     (int)std::min<int64_t>(G, (int64_t)cus), d_counts, st);
    }
    GPM_LAUNCH_CHECK("k_batch<1024>");
    const int lo256 = cfg->tiers >= 2 ? 128 : -1;
    {
        Span sp("k_batch<256>", st);
        launch_small<256>(nt, g, d_voff, b, lo256, k, b.tcur + 1, small, d_counts, st);
    }
    GPM_LAUNCH_CHECK("k_batch<256>");
    if (cfg->tiers >= 2) {
        const int lo128 = cfg->tiers >= 3 ? 64 : -1;
        {
            Span sp("k_batch<128>", st);
            launch_small<128>(nt, g, d_voff, b, lo128, k, b.tcur + 2, small, d_counts, st);
        }
        GPM_LAUNCH_CHECK("k_batch<128>");
    }
    if (cfg->tiers >= 3) {
        {
            Span sp("k_batch<64>", st);
            launch_small<64>(nt, g, d_voff, b, -1, k, b.tcur + 3, small, d_counts, st);
        }
        GPM_LAUNCH_CHECK("k_batch<64>");
    }
    return GPM_OK;
}

gpm_status batch_autotune(const gpm_graph *g, const int32_t *d_voff, int32_t G, int32_t k,
                          void *ws, uint64_t ws_bytes, unsigned long long *d_counts,
                          hipStream_t st, int32_t reps, gpm_batch_config *best,
                          float *best_ms) {
    std::vector<gpm_batch_config> cands;
    for (int nt : {64, 128, 256})
        for (int tiers : {1, 2, 3})
            for (int bpc : {4, 8, 16, 32}) cands.push_back({nt, tiers, bpc, 0});
    hipEvent_t e0, e1;
    GPM_HIP(hipEventCreate(&e0));
    GPM_HIP(hipEventCreate(&e1));
    float best_t = -1.0f;
    gpm_status rc = GPM_OK;
    for (const gpm_batch_config &c : cands) {
        rc = batch_run(g, d_voff, G, k, &c, ws, ws_bytes, d_counts, st);   // warm-up
        if (rc) break;
        hipError_t he = hipEventRecord(e0, st);
        for (int r = 0; r < reps && !rc && he == hipSuccess; r++)
            rc = batch_run(g, d_voff, G, k, &c, ws, ws_bytes, d_counts, st);
        if (rc) break;
        if (he == hipSuccess) he = hipEventRecord(e1, st);
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        if (he != hipSuccess) {
            rc = hip_fail(he, "autotune timing");
            break;
        }
        ms /= (float)reps;
        if (best_t < 0.0f || ms < best_t) {
            best_t = ms;
            *best = c;
        }
    }
    if (!rc) rc = batch_run(g, d_voff, G, k, best, ws, ws_bytes, d_counts, st);
    if (!rc && hipStreamSynchronize(st) != hipSuccess) rc = hip_fail(hipGetLastError(), "autotune");
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (best_ms) *best_ms = best_t;
    return rc;
}

// ------------------------------------------------- static scratch entry --
// gpm_batch_motif_count_static: the batch's work area (histogram, tier
// cursors, the largest-first graph order: batch_workspace_bytes) lives in a
// file-scope device array instead of a caller workspace, so the call makes
// no allocation of any kind.  Each device holds its own copy of the array;
// its address is looked up once per device (the host-side name of a
// __device__ array is not a device address) and kept.  Every call on a
// device uses that device's copy: calls that overlap in time on one device
// race on it.  batch_run clears what must start at zero (histogram, cursors)
// with fill kernels before use, so whatever an earlier call left there does
// not matter.
static __device__ __align__(256) unsigned char scratch[GPM_BATCH_STATIC_SCRATCH_BYTES];
static_assert((kWsHead + GPM_BATCH_STATIC_MAX_GRAPHS) * 4 <= GPM_BATCH_STATIC_SCRATCH_BYTES &&
                  (kWsHead + GPM_BATCH_STATIC_MAX_GRAPHS + 1) * 4 > GPM_BATCH_STATIC_SCRATCH_BYTES,
              "GPM_BATCH_STATIC_MAX_GRAPHS is the largest batch the static scratch holds");

namespace {

gpm_status static_scratch(void **out) {
    int dev = 0;
    GPM_HIP(hipGetDevice(&dev));
    static std::mutex mu;
    static std::map<int, void *> ptrs;
    std::lock_guard<std::mutex> lock(mu);
    auto it = ptrs.find(dev);
    if (it != ptrs.end()) {
        *out = it->second;
        return GPM_OK;
    }
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    ptrs[dev] = p;
    *out = p;
    return GPM_OK;
}

}  // namespace

gpm_status batch_run_static(const gpm_graph *g, const int32_t *d_voff, int32_t G, int32_t k,
                            unsigned long long *d_counts, hipStream_t st) {
    uint64_t need = 0;
    batch_workspace_bytes(G, k, &need);
    if (need > GPM_BATCH_STATIC_SCRATCH_BYTES)
        return fail(GPM_OUT_OF_MEMORY,
                    "batch too large for the static scratch: G = " + std::to_string(G) +
                        " needs " + std::to_string(need) + " bytes, the static scratch holds " +
                        std::to_string((uint64_t)GPM_BATCH_STATIC_SCRATCH_BYTES) +
                        " (at most GPM_BATCH_STATIC_MAX_GRAPHS graphs)");
    void *ws = nullptr;
    gpm_status rc = static_scratch(&ws);
    if (rc) return rc;
    gpm_batch_config cfg;
    batch_default_config(&cfg);
    spans_suppress(true);
    rc = batch_run(g, d_voff, G, k, &cfg, ws, GPM_BATCH_STATIC_SCRATCH_BYTES, d_counts, st);
    spans_suppress(false);
    return rc;
}

}  // namespace gpm
