// Subgraph listing (Section 2, problem 3; edge-induced embeddings) of the
// diamond and the 4-cycle, counting or listing.
//
// Diamond: its diagonal is the only edge whose two ends both have degree 3
// inside it, so the diamonds are exactly the pairs {c, d} of common
// neighbours of each edge (a, b): C(T_ab, 2) per edge, summed (the local
// count of Section 5).  Matching order (Appendix B.3, triangle first): the
// edge (a, b), then c and d from N(a) ∩ N(b) with c < d (Appendix B.1
// partial order of the two symmetric tips).  Listing walks one flattened
// index space holding every (edge, pair) with an atomic chunk cursor; a
// chunk recomputes its edge's common-neighbour list by a wave-cooperative
// intersection (lanes binary-search the longer list) into per-wave scratch.
//
// 4-cycle: see c4.hip.
#include "gpm_internal.h"

#include <algorithm>
#include <cmath>

namespace gpm {

gpm_status clique_workspace_bytes(const gpm_graph *g, int32_t k, bool list, uint64_t *bytes);
gpm_status triangle_arc_counts(const gpm_graph *g, void *ws, uint64_t ws_bytes, uint32_t *te,
                               unsigned long long *tri, hipStream_t st);
gpm_status c4_workspace_bytes(const gpm_graph *g, bool list, uint64_t *bytes);
gpm_status c4_run(const gpm_graph *g, bool list, void *ws, uint64_t ws_bytes,
                  unsigned long long *out128, int32_t *d_buf, uint64_t cap,
                  unsigned long long *d_result, hipStream_t st,
                  const uint32_t *tsym = nullptr, unsigned long long *cs = nullptr);

namespace {

typedef unsigned __int128 u128;

constexpr int kBlock = 256;
constexpr int kWPB = kBlock / kWave;
constexpr int64_t kPairChunk = 1 << 16;
constexpr int kPairUnroll = 8;   // consecutive pairs per lane when listing

__device__ __forceinline__ int lower_bound_i32(const int32_t *a, int n, int32_t x) {
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ int64_t last_le_i64(const int64_t *a, int64_t n, int64_t x) {
    int64_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (a[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint64_t edge_code(int32_t a, int32_t b) {
    const uint32_t lo = (uint32_t)min(a, b), hi = (uint32_t)max(a, b);
    return ((uint64_t)lo << 32) | hi;
}

// sum over arcs of C(T_e, 2), 128 bits.
__global__ void __launch_bounds__(kBlock) k_diamond_sum(const uint32_t *te, int64_t m,
                                                        unsigned long long *out) {
    int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    uint64_t s = 0;
    for (; e < m; e += stride) {
        const uint64_t t = te[e];
        s += t * (t - (t > 0)) / 2;
    }
    s = wave_sum(s);
    if (lane_id() == 0 && s) atomic_add_u128(out, (u128)s);
}

__global__ void k_copy_low(const unsigned long long *src, unsigned long long *dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) dst[0] = src[0];
}

// Active arcs (T_e >= 2) and their pair counts.
__global__ void k_pair_flag(const uint32_t *te, int64_t m, int32_t *flag) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; e < m; e += stride) flag[e] = te[e] >= 2 ? 1 : 0;
}

__global__ void k_pair_compact(const uint32_t *te, const int32_t *pos, int64_t m, int32_t *act,
                               int64_t *npairs) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; e < m; e += stride) {
        const uint64_t t = te[e];
        if (t >= 2) {
            act[pos[e]] = (int32_t)e;
            npairs[pos[e]] = (int64_t)(t * (t - 1) / 2);
        }
    }
}

struct Out {
    unsigned long long *slot_ctr;
    int32_t *buf;
    uint64_t cap;
};

// Diamond listing over the flattened (edge, pair) space.
__global__ void __launch_bounds__(kBlock) k_diamond_list(const int32_t *__restrict__ off,
                                                         const int32_t *__restrict__ adj,
                                                         const int32_t *__restrict__ dag_src,
                                                         const int32_t *__restrict__ dag_adj,
                                                         const int32_t *__restrict__ act,
                                                         const int64_t *__restrict__ ppre,
                                                         const int32_t *__restrict__ nact_p,
                                                         uint32_t *cursor, int32_t *scratch,
                                                         int32_t maxdeg, Out out,
                                                         unsigned long long *result) {
    const int lane = lane_id();
    const int64_t wave_gid = (int64_t)blockIdx.x * kWPB + threadIdx.x / kWave;
    int32_t *com = scratch + wave_gid * (int64_t)maxdeg;
    const int32_t nact = *nact_p;
    const int64_t total = ppre[nact];
    const uint64_t nchunks = (uint64_t)((total + kPairChunk - 1) / kPairChunk);
    uint64_t cached = 0, count = 0, hsum = 0;
    for (;;) {
        uint32_t c = 0;
        if (lane == 0) c = atomicAdd(cursor, 1u);
        c = __shfl(c, 0, 64);
        if (c >= nchunks) break;
        int64_t p = (int64_t)c * kPairChunk;
        const int64_t p1 = min(p + kPairChunk, total);
        int64_t ai = last_le_i64(ppre, nact + 1, p);
        while (p < p1) {
            const int64_t q0 = p - ppre[ai], q1 = min(p1, ppre[ai + 1]) - ppre[ai];
            const int32_t e = act[ai];
            const int32_t a = dag_src[e], b = dag_adj[e];
            // common neighbours of a and b, ascending
            const int32_t *na = adj + off[a], *nb = adj + off[b];
            int32_t da = off[a + 1] - off[a], db = off[b + 1] - off[b];
            if (da > db) {
                const int32_t *t = na; na = nb; nb = t;
                const int32_t td = da; da = db; db = td;
            }
            int32_t t = 0;
            for (int32_t i0 = 0; i0 < da; i0 += kWave) {
                const int32_t i = i0 + lane;
                bool hit = false;
                int32_t x = 0;
                if (i < da) {
                    x = na[i];
                    const int32_t k = lower_bound_i32(nb, db, x);
                    hit = k < db && nb[k] == x;
                }
                const uint64_t mask = __ballot(hit);
                if (hit) com[t + lanes_below(mask)] = x;
                t += __popcll(mask);
            }
            wave_sync();
            // each lane takes kPairUnroll consecutive pairs (i, j), i < j,
            // of the common neighbours: it decodes the first and steps
            for (int64_t qb = q0; qb < q1; qb += kWave * kPairUnroll) {
                const int64_t qs = qb + (int64_t)lane * kPairUnroll;
                int32_t i = 0, j = 0;
                if (qs < q1) {
                    // q = j (j - 1) / 2 + i; the single-precision root is off
                    // by at most one here
                    int64_t jj = (int64_t)((1.0f + sqrtf(1.0f + 8.0f * (float)qs)) * 0.5f);
                    while (jj * (jj - 1) / 2 > qs) jj--;
                    while ((jj + 1) * jj / 2 <= qs) jj++;
                    j = (int32_t)jj;
                    i = (int32_t)(qs - jj * (jj - 1) / 2);
                }
                int32_t cc[kPairUnroll], dd[kPairUnroll];
#pragma unroll
                for (int u = 0; u < kPairUnroll; u++) {
                    cc[u] = dd[u] = 0;
                    if (qs + u < q1) {
                        if (u > 0 && ++i == j) {
                            i = 0;
                            ++j;
                        }
                        cc[u] = com[i];
                        dd[u] = com[j];
                    }
                }
#pragma unroll
                for (int u = 0; u < kPairUnroll; u++) {
                    const bool active = qs + u < q1;
                    uint64_t h = 0;
                    if (active) {
                        uint64_t k[5] = {edge_code(a, b), edge_code(a, cc[u]), edge_code(a, dd[u]),
                                         edge_code(b, cc[u]), edge_code(b, dd[u])};
#pragma unroll
                        for (int x = 1; x < 5; x++)
#pragma unroll
                            for (int y = 4; y >= x; y--) {
                                const uint64_t lo = k[y - 1] < k[y] ? k[y - 1] : k[y];
                                const uint64_t hi = k[y - 1] < k[y] ? k[y] : k[y - 1];
                                k[y - 1] = lo;
                                k[y] = hi;
                            }
                        h = 5;
#pragma unroll
                        for (int x = 0; x < 5; x++) h = fmix64((h ^ k[x]) + 0x9E3779B97F4A7C15ull);
                    }
                    const uint64_t mask = __ballot(active);
                    if (!mask) continue;
                    const int n = __popcll(mask);
                    unsigned long long base = out.cap;
                    if (cached < out.cap) {
                        if (lane == 0) base = atomicAdd(out.slot_ctr, (unsigned long long)n);
                        base = __shfl(base, 0, 64);
                        cached = base + n;
                    }
                    if (active) {
                        count++;
                        hsum += h;
                        const uint64_t slot = base + lanes_below(mask);
                        if (slot < out.cap) {
                            int32_t *o = out.buf + slot * 4;
                            o[0] = a; o[1] = b; o[2] = cc[u]; o[3] = dd[u];
                        }
                    }
                }
            }
            wave_sync();
            p = min(p1, ppre[ai + 1]);
            ai++;
        }
    }
    count = wave_sum(count);
    hsum = wave_sum(hsum);
    if (lane == 0) {
        if (count) atomicAdd(&result[0], (unsigned long long)count);
        if (hsum) atomicAdd(&result[2], (unsigned long long)hsum);
    }
}

__global__ void k_finish(unsigned long long *result, const unsigned long long *slot_ctr,
                         uint64_t cap) {
    if (threadIdx.x == 0 && blockIdx.x == 0) result[1] = *slot_ctr < cap ? *slot_ctr : cap;
}

struct DiamondWs {
    uint32_t *ctl;
    unsigned long long *tri, *sum, *slot;
    uint32_t *te;
    int32_t *flag, *pos, *act;
    int64_t *npairs, *ppre, *scan_tmp;
    int32_t *scratch;
    int waves;
    void *tc;
    uint64_t tc_bytes, bytes;
};

DiamondWs diamond_layout(const gpm_graph *g, bool list, void *base) {
    DiamondWs W{};
    Carve c(base, ~0ull);
    const uint64_t m1 = (uint64_t)g->m + 1;
    W.ctl = c.take<uint32_t>(16);
    W.tri = c.take<unsigned long long>(2);
    W.sum = c.take<unsigned long long>(2);
    W.slot = c.take<unsigned long long>(2);
    W.te = c.take<uint32_t>(m1);
    if (list) {
        W.flag = c.take<int32_t>(m1);
        W.pos = c.take<int32_t>(m1);
        W.act = c.take<int32_t>(m1);
        W.npairs = c.take<int64_t>(m1);
        W.ppre = c.take<int64_t>(m1);
        W.scan_tmp = c.take<int64_t>(scan_tmp_words(m1));
        W.waves = persistent_blocks(kWPB, 4) * kWPB;
        W.scratch = c.take<int32_t>((uint64_t)W.waves * (uint64_t)std::max(1, g->max_degree));
    }
    clique_workspace_bytes(g, 3, false, &W.tc_bytes);
    W.tc = c.take<char>(W.tc_bytes);
    W.bytes = c.used;
    return W;
}

unsigned grid_for(int64_t items, int per_block, int cap_per_cu) {
    int64_t b = (items + per_block - 1) / per_block;
    int64_t cap = (int64_t)cu_count() * cap_per_cu;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

gpm_status diamond_run(const gpm_graph *g, bool list, void *ws, uint64_t ws_bytes,
                       unsigned long long *d_count, int32_t *d_buf, uint64_t cap,
                       unsigned long long *d_result, hipStream_t st) {
    DiamondWs W = diamond_layout(g, list, ws);
    if (W.bytes > ws_bytes) return fail(GPM_OUT_OF_MEMORY, "workspace smaller than required");
    const int64_t m = g->m;
    GPM_HIP(fill_u32(W.ctl, 0, 16, st));
    GPM_HIP(fill_u32(W.tri, 0, 4, st));
    GPM_HIP(fill_u32(W.sum, 0, 4, st));
    GPM_HIP(fill_u32(W.slot, 0, 4, st));
    if (m > 0) GPM_HIP(fill_u32(W.te, 0, (uint64_t)m, st));
    gpm_status rc = triangle_arc_counts(g, W.tc, W.tc_bytes, W.te, W.tri, st);
    if (rc) return rc;
    if (!list) {
        if (m > 0) {
            Span sp("k_diamond_sum", st);
            hipLaunchKernelGGL(k_diamond_sum, dim3(grid_for(m, kBlock, 8)), dim3(kBlock), 0, st,
                               W.te, m, W.sum);
        }
        GPM_LAUNCH_CHECK("k_diamond_sum");
        hipLaunchKernelGGL(k_copy_low, dim3(1), dim3(64), 0, st, W.sum, d_count);
        GPM_LAUNCH_CHECK("k_copy_low");
        return GPM_OK;
    }
    GPM_HIP(fill_u32(d_result, 0, 6, st));
    GPM_HIP(fill_u32(W.npairs, 0, 2 * ((uint64_t)m + 1), st));
    hipLaunchKernelGGL(k_pair_flag, dim3(grid_for(m, 256, 8)), dim3(256), 0, st, W.te, m, W.flag);
    GPM_HIP(exclusive_scan_i32(W.flag, W.pos, (uint64_t)m, W.scan_tmp, st));
    hipLaunchKernelGGL(k_pair_compact, dim3(grid_for(m, 256, 8)), dim3(256), 0, st, W.te, W.pos,
                       m, W.act, W.npairs);
    GPM_LAUNCH_CHECK("k_pair_compact");
    GPM_HIP(exclusive_scan_64(W.npairs, W.ppre, (uint64_t)m, W.scan_tmp, st));
    Out out{W.slot, d_buf, d_buf ? cap : 0};
    {
        Span sp("k_diamond_list", st);
        hipLaunchKernelGGL(k_diamond_list, dim3((unsigned)(W.waves / kWPB)), dim3(kBlock), 0, st,
                           g->off, g->adj, g->dag_src, g->dag_adj, W.act, W.ppre,
                           W.pos + m, W.ctl + 0, W.scratch, std::max(1, g->max_degree), out,
                           d_result);
    }
    GPM_LAUNCH_CHECK("k_diamond_list");
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(64), 0, st, d_result, W.slot, d_buf ? cap : 0);
    GPM_LAUNCH_CHECK("k_finish");
    return GPM_OK;
}

struct C4CountWs {
    unsigned long long *sum;
    void *c4;
    uint64_t c4_bytes, bytes;
};

C4CountWs c4count_layout(const gpm_graph *g, bool list, void *base) {
    C4CountWs W{};
    Carve c(base, ~0ull);
    W.sum = c.take<unsigned long long>(2);
    c4_workspace_bytes(g, list, &W.c4_bytes);
    W.c4 = c.take<char>(W.c4_bytes);
    W.bytes = c.used;
    return W;
}

}  // namespace

gpm_status sl_workspace_bytes(const gpm_graph *g, int32_t plan, bool list, uint64_t *bytes) {
    if (plan == GPM_PLAN_SL_DIAMOND) {
        *bytes = diamond_layout(g, list, nullptr).bytes;
        return GPM_OK;
    }
    gpm_status rc = c4_workspace_bytes(g, list, bytes);
    if (rc) return rc;
    *bytes = c4count_layout(g, list, nullptr).bytes;
    return GPM_OK;
}

gpm_status sl_run(const gpm_graph *g, int32_t plan, bool list, void *ws, uint64_t ws_bytes,
                  unsigned long long *d_count, int32_t *d_buf, uint64_t cap,
                  unsigned long long *d_result, hipStream_t st) {
    if (plan == GPM_PLAN_SL_DIAMOND)
        return diamond_run(g, list, ws, ws_bytes, d_count, d_buf, cap, d_result, st);
    C4CountWs W = c4count_layout(g, list, ws);
    if (W.bytes > ws_bytes) return fail(GPM_OUT_OF_MEMORY, "workspace smaller than required");
    if (list) return c4_run(g, true, W.c4, W.c4_bytes, nullptr, d_buf, cap, d_result, st);
    GPM_HIP(fill_u32(W.sum, 0, 4, st));
    gpm_status rc = c4_run(g, false, W.c4, W.c4_bytes, W.sum, nullptr, 0, nullptr, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_copy_low, dim3(1), dim3(64), 0, st, W.sum, d_count);
    GPM_LAUNCH_CHECK("k_copy_low");
    return GPM_OK;
}

// Column permutation of the written rows of a 4-vertex listing:
// row'[p] = row[perm[p]] for the first min(result[1], cap) rows (result[1]
// = rows written, set by the listing before this runs on the stream).
struct Perm4 {
    int32_t p[4];
};

__global__ void k_permute_rows4(int32_t *buf, uint64_t cap, const unsigned long long *result,
                                Perm4 perm) {
    const uint64_t w = result[1] < cap ? result[1] : cap;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < w; i += stride) {
        int4 *r = reinterpret_cast<int4 *>(buf + 4 * i);
        const int4 x = *r;
        const int32_t v[4] = {x.x, x.y, x.z, x.w};
        *r = make_int4(v[perm.p[0]], v[perm.p[1]], v[perm.p[2]], v[perm.p[3]]);
    }
}

gpm_status permute_rows4(int32_t *buf, uint64_t cap, const unsigned long long *result,
                         const int32_t perm[4], hipStream_t st) {
    if (cap == 0) return GPM_OK;
    Perm4 p;
    for (int i = 0; i < 4; i++) p.p[i] = perm[i];
    const unsigned blocks = (unsigned)std::min<uint64_t>((cap + 255) / 256, (uint64_t)cu_count() * 8);
    hipLaunchKernelGGL(k_permute_rows4, dim3(blocks), dim3(256), 0, st, buf, cap, result, p);
    GPM_LAUNCH_CHECK("k_permute_rows4");
    return GPM_OK;
}

}  // namespace gpm
