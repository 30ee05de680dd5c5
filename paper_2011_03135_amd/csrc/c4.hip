// 4-cycles (every edge set forming a 4-cycle, i.e. edge-induced embeddings;
// Section 2, subgraph listing), counted and listed from each cycle's
// highest-ranked vertex x in the degree order (the orientation order of
// Appendix B.2).
//
// Matching order (Appendix B.3): x first, then its lower-ranked neighbour y
// (wedge x - y), then z, a neighbour of y ranked below x (z != x), then the
// second middle y' with y' < y adjacent to both x and z.  The partial orders
// that leave one copy of each cycle (Appendix B.1): x above every other
// cycle vertex, and the two middles ordered.  Grouping the wedges of one
// apex x by their end z gives c(x, z) middles and C(c(x, z), 2) cycles.
//
// Counting forms sum C(c, 2) incrementally: each new wedge to z adds the
// number of earlier ones.  Listing groups each apex's wedges by z and emits
// every pair of middles.
//   light apex (wedge work <= kLightW): one wave, wedges in LDS;
//   heavy apex: tasks (x, part p) for z in the part's id range, dense LDS
//   counters over the range; each N(y) is entered at the part through a
//   part-major table of per-vertex segments, or by binary search when the
//   table would be too large.
#include "gpm_internal.h"

#include <algorithm>

namespace gpm {

namespace {

typedef unsigned __int128 u128;

constexpr int kBlock = 256;
constexpr int kWPB = kBlock / kWave;
constexpr int kLightW = 512;         // wedge work of a light apex
constexpr int kHashSlots = 1024;     // per-wave LDS hash (load <= 1/2)
constexpr int kPartZ = 8192;         // z-range per heavy task (LDS counters)
constexpr int kYChunk = kBlock;      // in-neighbours staged per round
constexpr int kListBlocks = 512;     // workgroups of the heavy listing kernel
constexpr int kWedgeCap = 1 << 18;   // per-workgroup wedge buffer (>= max degree)

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int lower_bound_i32(const int32_t *a, int n, int32_t x) {
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ int last_le_i32(const int32_t *a, int n, int32_t x) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (a[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ void k_degrees(const int32_t *off, int32_t n, int32_t *deg) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) deg[i] = off[i + 1] - off[i];
}

// adeg[e] = degree of the end of arc e, so the rank test of a wedge's end
// is a coalesced read next to the arc instead of a gather.
__global__ void k_arc_deg(const int32_t *adj, const int32_t *deg, int64_t arcs, int32_t *adeg) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < arcs; i += stride) adeg[i] = deg[adj[i]];
}

enum C4Class : int { C4_NONE = 0, C4_LIGHT = 1, C4_HEAVY = 2 };

// Class of apex x by its wedge work, the sum of d(y) over in-neighbours y.
__global__ void __launch_bounds__(kBlock) k_c4_work(const int32_t *__restrict__ off,
                                                    const int32_t *__restrict__ adj,
                                                    const int32_t *__restrict__ deg, int32_t n,
                                                    int32_t *cls) {
    const int lane = lane_id();
    const int64_t wave0 = (int64_t)blockIdx.x * kWPB + threadIdx.x / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * kWPB;
    for (int64_t r = wave0; r < n; r += nwaves) {
        const int32_t x = (int32_t)r, s = off[x], dx = off[x + 1] - s;
        int64_t w = 0;
        int32_t ny = 0;
        for (int32_t i = lane; i < dx; i += kWave) {
            const int32_t y = adj[s + i], dy = deg[y];
            if (rank_less(dy, y, dx, x)) {
                w += dy;
                ny++;
            }
        }
        w = wave_sum(w);
        ny = wave_sum(ny);
        if (lane == 0) cls[x] = (ny < 2) ? C4_NONE : (w <= kLightW ? C4_LIGHT : C4_HEAVY);
    }
}

__global__ void k_flag_eq(const int32_t *cls, int32_t n, int32_t want, int32_t *flag) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) flag[i] = cls[i] == want ? 1 : 0;
}

__global__ void k_compact_eq(const int32_t *cls, const int32_t *pos, int32_t n, int32_t want,
                             int32_t *list) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride)
        if (cls[i] == want) list[pos[i]] = (int32_t)i;
}

// ------------------------------------------------------------- emission ---

// Wave-cooperative listing output: a shared slot counter hands out buffer
// rows while the buffer has room; totals and checksums are per lane.
struct Emitter {
    unsigned long long *slot_ctr;
    int32_t *buf;
    uint64_t cap;
    uint64_t cached;   // wave-uniform: last slot counter value seen
    uint64_t count;    // per lane
    uint64_t hsum;     // per lane
};

__device__ __forceinline__ uint64_t edge_code(int32_t a, int32_t b) {
    const uint32_t lo = (uint32_t)min(a, b), hi = (uint32_t)max(a, b);
    return ((uint64_t)lo << 32) | hi;
}

// Hash of an embedding's ascending key (see gpm_list in gpm.h).
template <int L>
__device__ __forceinline__ uint64_t key_hash(uint64_t (&k)[L]) {
#pragma unroll
    for (int i = 1; i < L; i++)
#pragma unroll
        for (int j = L - 1; j >= i; j--) {
            const uint64_t a = k[j - 1], b = k[j];
            k[j - 1] = a < b ? a : b;
            k[j] = a < b ? b : a;
        }
    uint64_t h = (uint64_t)L;
#pragma unroll
    for (int i = 0; i < L; i++) h = fmix64((h ^ k[i]) + 0x9E3779B97F4A7C15ull);
    return h;
}

// Must be reached by the whole wave; `active` lanes emit (a, b, c, d).
__device__ __forceinline__ void emit4(Emitter &em, bool active, int32_t a, int32_t b, int32_t c,
                                      int32_t d, uint64_t h) {
    const uint64_t mask = __ballot(active);
    if (!mask) return;
    const int cnt = __popcll(mask);
    unsigned long long base = em.cap;
    if (em.cached < em.cap) {
        if (lane_id() == 0) base = atomicAdd(em.slot_ctr, (unsigned long long)cnt);
        base = __shfl(base, 0, 64);
        em.cached = base + cnt;
    }
    if (active) {
        em.count++;
        em.hsum += h;
        const uint64_t slot = base + lanes_below(mask);
        if (slot < em.cap) {
            int32_t *o = em.buf + slot * 4;
            o[0] = a; o[1] = b; o[2] = c; o[3] = d;
        }
    }
}

__device__ __forceinline__ void emit_c4(Emitter &em, bool active, int32_t x, int32_t y1,
                                        int32_t z, int32_t y2) {
    uint64_t h = 0;
    if (active) {
        uint64_t k[4] = {edge_code(x, y1), edge_code(y1, z), edge_code(z, y2), edge_code(y2, x)};
        h = key_hash<4>(k);
    }
    emit4(em, active, x, y1, z, y2, h);
}

__device__ __forceinline__ void emitter_flush(Emitter &em, unsigned long long *result) {
    const uint64_t c = wave_sum(em.count), h = wave_sum(em.hsum);
    if (lane_id() == 0) {
        if (c) atomicAdd(&result[0], (unsigned long long)c);
        if (h) atomicAdd(&result[2], (unsigned long long)h);
    }
}

// -------------------------------------------------------------- counting ---

__device__ __forceinline__ uint32_t hash_slot(int32_t z) {
    return ((uint32_t)z * 0x9E3779B1u) >> 22;   // 10 bits -> kHashSlots
}

// Stages apex x's in-neighbours y (ranked below x): base[j] = off[y_j],
// pre[j+1] = prefix of d(y_j), ylist[j] = y_j, arcs[j] = the arc x -> y_j.
// Returns the wedge work.
__device__ __forceinline__ int32_t stage_in(const int32_t *__restrict__ off,
                                            const int32_t *__restrict__ adj,
                                            const int32_t *__restrict__ deg, int32_t x, int32_t s,
                                            int32_t dx, int32_t *pre, int32_t *base, int32_t *ylist,
                                            int32_t &ny, int32_t *arcs = nullptr) {
    const int lane = lane_id();
    int32_t carry = 0;
    ny = 0;
    for (int32_t i0 = 0; i0 < dx; i0 += kWave) {
        const int32_t i = i0 + lane;
        int32_t y = 0, dy = 0;
        bool in = false;
        if (i < dx) {
            y = adj[s + i];
            dy = deg[y];
            in = rank_less(dy, y, dx, x);
        }
        const uint64_t mask = __ballot(in);
        const int32_t p = ny + lanes_below(mask);
        const int32_t inc = wave_incl_scan(in ? dy : 0);
        if (in) {
            base[p] = off[y];
            pre[p + 1] = carry + inc;
            if (ylist) ylist[p] = y;
            if (arcs) arcs[p] = s + i;
        }
        carry += __shfl(inc, 63, 64);
        ny += __popcll(mask);
    }
    if (lane == 0) pre[0] = 0;
    wave_sync();
    return carry;
}

// Sums over the 4-cycles, from the wedges once their groups are complete:
// a wedge x - y - z whose group holds c wedges lies on c - 1 cycles, and
// each cycle has two wedges (middles y and y') from its apex x to its
// opposite vertex z, so
//   sum over cycles of (d_x + d_y + d_z + d_y')  is half the sum over
//       wedges of (c - 1)(d_x + d_z + 2 d_y)                (cs[0..1], doubled)
//   sum over cycles of the triangle counts of its four edges  is the sum
//       over wedges of (c - 1)(T_xy + T_yz)                  (cs[2..3])
// (tsym: triangle count per arc of the symmetric CSR).
struct CycleSums {
    uint64_t deg2 = 0, tri = 0;
    __device__ __forceinline__ void add(uint32_t c, uint32_t dx, uint32_t dy, uint32_t dz,
                                        uint32_t txy, uint32_t tyz) {
        const uint64_t k = c - 1u;
        deg2 += k * ((uint64_t)dx + dz + 2ull * dy);
        tri += k * ((uint64_t)txy + tyz);
    }
    __device__ __forceinline__ void flush(unsigned long long *cs) {
        const u128 a = wave_sum_u128((u128)deg2), b = wave_sum_u128((u128)tri);
        if (lane_id() == 0) {
            if (a) atomic_add_u128(cs, a);
            if (b) atomic_add_u128(cs + 2, b);
        }
    }
};

// Light apexes: one wave each, LDS hash z -> count, wedge by wedge.  With
// CS, a second walk over the apex's wedges adds the cycle sums.
template <bool CS>
__global__ void __launch_bounds__(kBlock) k_c4_light(const int32_t *__restrict__ off,
                                                     const int32_t *__restrict__ adj,
                                                     const int32_t *__restrict__ deg,
                                                     const int32_t *__restrict__ adeg,
                                                     const int32_t *__restrict__ list,
                                                     const int32_t *__restrict__ count_p,
                                                     unsigned long long *out,
                                                     const uint32_t *__restrict__ tsym,
                                                     unsigned long long *cs) {
    __shared__ int32_t s_key[kWPB][kHashSlots];
    __shared__ uint32_t s_cnt[kWPB][kHashSlots];
    __shared__ int32_t s_pre[kWPB][kLightW + 1];
    __shared__ int32_t s_base[kWPB][kLightW];
    __shared__ int32_t s_arc[CS ? kWPB : 1][CS ? kLightW : 1];
    const int lane = lane_id(), wib = threadIdx.x / kWave;
    int32_t *key = s_key[wib], *pre = s_pre[wib], *base = s_base[wib];
    int32_t *arcs = CS ? s_arc[wib] : nullptr;
    uint32_t *cnt = s_cnt[wib];
    const int32_t count = *count_p;
    const int64_t wave0 = (int64_t)blockIdx.x * kWPB + wib;
    const int64_t nwaves = (int64_t)gridDim.x * kWPB;
    for (int i = lane; i < kHashSlots; i += kWave) { key[i] = -1; cnt[i] = 0; }
    uint64_t acc = 0;
    CycleSums sums;
    for (int64_t r = wave0; r < count; r += nwaves) {
        const int32_t x = list[r], s = off[x], dx = off[x + 1] - s;
        int32_t ny;
        const int32_t W = stage_in(off, adj, deg, x, s, dx, pre, base, nullptr, ny, arcs);
        for (int32_t qb = 0; qb < W; qb += kWave) {
            const int32_t q = qb + lane;
            if (q < W) {
                const int32_t j = last_le_i32(pre, ny + 1, q);
                const int32_t e = base[j] + (q - pre[j]);
                const int32_t z = adj[e];
                if (rank_less(adeg[e], z, dx, x)) {
                    uint32_t h = hash_slot(z);
                    for (;;) {
                        int32_t k = key[h];
                        if (k == -1) {
                            k = atomicCAS(&key[h], -1, z);
                            if (k == -1) k = z;
                        }
                        if (k == z) {
                            acc += atomicAdd(&cnt[h], 1u);
                            break;
                        }
                        h = (h + 1) & (kHashSlots - 1);
                    }
                }
            }
        }
        wave_sync();
        if (CS) {
            for (int32_t qb = 0; qb < W; qb += kWave) {
                const int32_t q = qb + lane;
                if (q < W) {
                    const int32_t j = last_le_i32(pre, ny + 1, q);
                    const int32_t e = base[j] + (q - pre[j]);
                    const int32_t z = adj[e];
                    if (rank_less(adeg[e], z, dx, x)) {
                        uint32_t h = hash_slot(z);
                        while (key[h] != z) h = (h + 1) & (kHashSlots - 1);
                        sums.add(cnt[h], (uint32_t)dx, (uint32_t)(pre[j + 1] - pre[j]),
                                 (uint32_t)adeg[e], tsym[arcs[j]], tsym[e]);
                    }
                }
            }
            wave_sync();
        }
        for (int i = lane; i < kHashSlots; i += kWave)
            if (key[i] != -1) { key[i] = -1; cnt[i] = 0; }
        wave_sync();
    }
    acc = wave_sum(acc);
    if (lane == 0 && acc) atomic_add_u128(out, (u128)acc);
    if (CS) sums.flush(cs);
}

// Heavy apexes, counting.  Task (z-part p, apex x), part-major so that the
// tasks running together share one part's table row and degree slice.  The
// block keeps a dense LDS counter per z of the part; for each in-neighbour
// y of x it takes the segment of N(y) inside the part (from the part table,
// else by binary search in N(y)), and the block walks the concatenated
// segments, one wedge per lane: each wedge to a z ranked below x adds the
// count of earlier wedges to that z (the C(c, 2) sum).  A counter
// c(x, z) never exceeds deg(z), and z, ranked below x, is never the
// top-ranked vertex, so when at most one vertex has a degree above 65535
// the counters are 16 bits, two to a word, and a part spans 65536 ids
// instead of 32768: half the tasks, segments twice as long.
constexpr int kCountWords = 32768;   // LDS counter words of a counting task (128 KiB)
constexpr int kHeavyNT = 1024;
constexpr int kSegMaxParts = 256;    // part table only for graphs of at most 256 parts
constexpr uint64_t kSegMaxBytes = 2ull << 30;

// Part table: seg[p * n + y] = {first arc of N(y) with end >= p * zpart,
// number of arcs of N(y) with end in part p}.
__global__ void __launch_bounds__(kBlock) k_c4_seg(const int32_t *__restrict__ off,
                                                   const int32_t *__restrict__ adj, int32_t n,
                                                   int32_t nparts, int32_t zpart, int2 *seg) {
    __shared__ int32_t s_bnd[kWPB][kSegMaxParts + 1];
    const int lane = lane_id();
    int32_t *bnd = s_bnd[threadIdx.x / kWave];
    const int64_t wave0 = (int64_t)blockIdx.x * kWPB + threadIdx.x / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * kWPB;
    for (int64_t y = wave0; y < n; y += nwaves) {
        const int32_t s = off[y], d = off[y + 1] - s;
        for (int32_t i = lane; i < d; i += kWave) {
            const int32_t pc = adj[s + i] / zpart;
            const int32_t pp = i == 0 ? -1 : adj[s + i - 1] / zpart;
            for (int32_t q = pp + 1; q <= pc; q++) bnd[q] = i;
        }
        const int32_t plast = d > 0 ? adj[s + d - 1] / zpart : -1;
        for (int32_t q = plast + 1 + lane; q <= nparts; q += kWave) bnd[q] = d;
        wave_sync();
        for (int32_t q = lane; q < nparts; q += kWave)
            seg[(int64_t)q * n + y] = make_int2(s + bnd[q], bnd[q + 1] - bnd[q]);
        wave_sync();
    }
}

// Last j in [lo, hi) with pre[j] <= q, given pre[lo] <= q.
__device__ __forceinline__ int32_t seg_of(const int32_t *pre, int32_t lo, int32_t hi, int32_t q) {
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (pre[mid] <= q) lo = mid; else hi = mid;
    }
    return lo;
}

//
// With CS, a second walk over the task's wedges, once its counters are
// complete, adds the cycle sums (CycleSums above).
template <bool CS>
__global__ void __launch_bounds__(kHeavyNT) k_c4_heavy(const int32_t *__restrict__ off,
                                                       const int32_t *__restrict__ adj,
                                                       const int32_t *__restrict__ adeg,
                                                       const int32_t *__restrict__ list,
                                                       const int32_t *__restrict__ count_p,
                                                       int32_t n, int32_t nparts, int32_t narrow,
                                                       const int2 *__restrict__ seg,
                                                       uint32_t *cursor, unsigned long long *out,
                                                       const uint32_t *__restrict__ tsym,
                                                       unsigned long long *cs) {
    constexpr int NW = kHeavyNT / kWave;
    __shared__ uint32_t cnt[kCountWords];
    __shared__ int32_t s_pre[kHeavyNT + 1];
    __shared__ int32_t s_off[kHeavyNT];    // segment start arc minus its pair prefix
    __shared__ int32_t s_sum[NW];
    __shared__ uint32_t s_dy[CS ? kHeavyNT : 1];    // d(y) of each segment
    __shared__ uint32_t s_txy[CS ? kHeavyNT : 1];   // triangles on the arc x -> y
    __shared__ uint32_t s_task;
    const int tid = threadIdx.x, lane = lane_id(), wid = tid / kWave;
    const int32_t nheavy = *count_p;
    const uint64_t ntasks = (uint64_t)nheavy * (uint64_t)nparts;
    uint64_t acc = 0;
    CycleSums sums;
    const int32_t zpart = narrow ? 2 * kCountWords : kCountWords;
    for (int i = tid; i < kCountWords; i += kHeavyNT) cnt[i] = 0;
    for (;;) {
        if (tid == 0) s_task = atomicAdd(cursor, 1u);
        __syncthreads();
        const uint64_t t = s_task;
        __syncthreads();
        if (t >= ntasks) break;
        const int32_t part = (int32_t)(t / (uint64_t)nheavy);
        const int32_t x = list[t % (uint64_t)nheavy];
        const int32_t z0 = part * zpart, z1 = z0 + zpart;
        const int32_t s = off[x], dx = off[x + 1] - s;
        for (int pass = 0; pass < (CS ? 2 : 1); pass++)
        for (int32_t c0 = 0; c0 < dx; c0 += kHeavyNT) {
            const int32_t i = c0 + tid;
            int32_t len[1] = {0}, start = 0;
            if (i < dx) {
                const int32_t y = adj[s + i], dy = adeg[s + i];
                if (rank_less(dy, y, dx, x)) {
                    if (seg) {
                        const int2 sg = seg[(int64_t)part * n + y];
                        start = sg.x;
                        len[0] = sg.y;
                    } else {
                        const int32_t oy = off[y];
                        const int32_t lo = lower_bound_i32(adj + oy, dy, z0);
                        const int32_t hi = lo + lower_bound_i32(adj + oy + lo, dy - lo, z1);
                        start = oy + lo;
                        len[0] = hi - lo;
                    }
                    if (CS) {
                        s_dy[tid] = (uint32_t)dy;
                        s_txy[tid] = tsym[s + i];
                    }
                }
            }
            block_prefix<kHeavyNT, 1>(len, kHeavyNT, s_pre, s_sum);   // ends with a barrier
            s_off[tid] = start - s_pre[tid];
            __syncthreads();
            const int32_t total = s_pre[kHeavyNT];
            // segments are short (a part of one list): each lane finds its
            // segment by binary search in the 64 segments after the previous
            // tile's last one, or beyond them
            const int32_t per_wave = ((total + NW - 1) / NW + kWave - 1) / kWave * kWave;
            const int32_t qa = min(total, wid * per_wave);
            const int32_t qz = min(total, qa + per_wave);
            int32_t j0 = qa < qz ? seg_of(s_pre, 0, kHeavyNT, qa) : 0;
            for (int32_t qb = qa; qb < qz; qb += kWave) {
                const int32_t q = qb + lane;
                int32_t j = j0;
                if (q < qz) {
                    const int32_t w = min(j0 + kWave, kHeavyNT);
                    j = s_pre[w] <= q ? seg_of(s_pre, w, kHeavyNT, q) : seg_of(s_pre, j0, w, q);
                    const int32_t e = s_off[j] + q;
                    const int32_t z = adj[e];
                    const int32_t dz = adeg[e];
                    if (rank_less(dz, z, dx, x)) {
                        const uint32_t zz = (uint32_t)(z - z0);
                        const uint32_t sh = narrow ? (zz & 1u) * 16u : 0u;
                        uint32_t *cw = narrow ? &cnt[zz >> 1] : &cnt[zz];
                        if (pass == 0) {
                            // each wedge to z adds the number of earlier ones
                            acc += narrow ? (atomicAdd(cw, 1u << sh) >> sh) & 0xffffu
                                          : atomicAdd(cw, 1u);
                        } else {
                            const uint32_t c = narrow ? (*cw >> sh) & 0xffffu : *cw;
                            sums.add(c, (uint32_t)dx, s_dy[j], (uint32_t)dz, s_txy[j], tsym[e]);
                        }
                    }
                }
                j0 = __shfl(j, kWave - 1, kWave);
            }
            __syncthreads();
        }
        for (int i = tid; i < kCountWords; i += kHeavyNT) cnt[i] = 0;
        __syncthreads();
    }
    acc = wave_sum(acc);
    if (lane == 0 && acc) atomic_add_u128(out, (u128)acc);
    if (CS) sums.flush(cs);
}

// --------------------------------------------------------------- listing ---

// Light apexes, listing: one wave gathers the apex's wedges (z, y) as 64-bit
// keys in LDS, sorts them, and emits every pair of middles of each z-run.
__global__ void __launch_bounds__(kBlock) k_c4_light_list(const int32_t *__restrict__ off,
                                                          const int32_t *__restrict__ adj,
                                                          const int32_t *__restrict__ deg,
                                                          const int32_t *__restrict__ list,
                                                          const int32_t *__restrict__ count_p,
                                                          Emitter em, unsigned long long *result) {
    __shared__ uint64_t s_keys[kWPB][kLightW];
    __shared__ int32_t s_pre[kWPB][kLightW + 1];
    __shared__ int32_t s_base[kWPB][kLightW + 1];   // also the pair prefix (nk + 1 entries)
    __shared__ int32_t s_y[kWPB][kLightW];
    const int lane = lane_id(), wib = threadIdx.x / kWave;
    uint64_t *keys = s_keys[wib];
    int32_t *pre = s_pre[wib], *base = s_base[wib], *ylist = s_y[wib];
    const int32_t count = *count_p;
    const int64_t wave0 = (int64_t)blockIdx.x * kWPB + wib;
    const int64_t nwaves = (int64_t)gridDim.x * kWPB;
    em.cached = 0;
    em.count = 0;
    em.hsum = 0;
    for (int64_t r = wave0; r < count; r += nwaves) {
        const int32_t x = list[r], s = off[x], dx = off[x + 1] - s;
        int32_t ny;
        const int32_t W = stage_in(off, adj, deg, x, s, dx, pre, base, ylist, ny);
        int32_t nk = 0;
        for (int32_t qb = 0; qb < W; qb += kWave) {
            const int32_t q = qb + lane;
            bool keep = false;
            uint64_t key = 0;
            if (q < W) {
                const int32_t j = last_le_i32(pre, ny + 1, q);
                const int32_t z = adj[base[j] + (q - pre[j])];
                keep = rank_less(deg[z], z, dx, x);
                key = ((uint64_t)(uint32_t)z << 32) | (uint32_t)ylist[j];
            }
            const uint64_t mask = __ballot(keep);
            if (keep) keys[nk + lanes_below(mask)] = key;
            nk += __popcll(mask);
        }
        int32_t P = 64;
        while (P < nk) P <<= 1;
        for (int32_t i = nk + lane; i < P; i += kWave) keys[i] = ~0ull;
        wave_sync();
        for (int32_t k = 2; k <= P; k <<= 1)
            for (int32_t j = k >> 1; j > 0; j >>= 1) {
                for (int32_t t = lane; t < P / 2; t += kWave) {
                    const int32_t i = (t / j) * 2 * j + (t % j), p = i + j;
                    const uint64_t a = keys[i], b = keys[p];
                    if ((a > b) == ((i & k) == 0)) {
                        keys[i] = b;
                        keys[p] = a;
                    }
                }
                wave_sync();
            }
        // pre[i] = start of i's z-run; base[i] = pairs (k, i), k in the run
        // before i, summed over positions before i
        int32_t carry_start = 0, carry_pairs = 0;
        for (int32_t i0 = 0; i0 < nk; i0 += kWave) {
            const int32_t i = i0 + lane;
            int32_t mine = (i < nk && (i == 0 || (keys[i] >> 32) != (keys[i - 1] >> 32))) ? i : -1;
            // inclusive max-scan of run starts
            int32_t run = mine;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int32_t other = __shfl_up(run, o, 64);
                if (lane >= o && other > run) run = other;
            }
            if (run < carry_start) run = carry_start;
            const int32_t pairs = i < nk ? i - run : 0;
            const int32_t inc = wave_incl_scan(pairs);
            if (i < nk) {
                pre[i] = run;
                base[i] = carry_pairs + inc - pairs;
            }
            carry_start = __shfl(run, 63, 64);
            carry_pairs += __shfl(inc, 63, 64);
        }
        if (lane == 0) base[nk] = carry_pairs;
        wave_sync();
        const int32_t npairs = carry_pairs;
        for (int32_t qb = 0; qb < npairs; qb += kWave) {
            const int32_t q = qb + lane;
            const bool active = q < npairs;
            int32_t y1 = 0, z = 0, y2 = 0;
            if (active) {
                const int32_t p = last_le_i32(base, nk + 1, q);   // second middle's position
                const int32_t i = pre[p] + (q - base[p]);
                z = (int32_t)(keys[p] >> 32);
                y1 = (int32_t)(uint32_t)keys[i];
                y2 = (int32_t)(uint32_t)keys[p];
            }
            emit_c4(em, active, x, y1, z, y2);
        }
        wave_sync();
    }
    emitter_flush(em, result);
}

// Heavy apexes, listing: workgroup per (apex, z-part); counts per z, then
// the part's wedges grouped by z in a per-workgroup HBM buffer (in z
// sub-ranges that fit it), then every pair of middles per z.
__global__ void __launch_bounds__(kBlock) k_c4_heavy_list(const int32_t *__restrict__ off,
                                                          const int32_t *__restrict__ adj,
                                                          const int32_t *__restrict__ deg,
                                                          const int32_t *__restrict__ list,
                                                          const int32_t *__restrict__ count_p,
                                                          int32_t nparts, uint32_t *cursor,
                                                          int32_t *wedge_buf, Emitter em,
                                                          unsigned long long *result) {
    __shared__ int32_t cnt[kPartZ + 1];     // counts, then prefix offsets
    __shared__ uint32_t cur[kPartZ];
    __shared__ int32_t s_pre[kYChunk + 1];
    __shared__ int32_t s_start[kYChunk];
    __shared__ int32_t s_sum[kWPB];
    __shared__ uint32_t s_task, s_z;
    const int tid = threadIdx.x, lane = lane_id(), wid = tid / kWave;
    const uint64_t ntasks = (uint64_t)(*count_p) * (uint64_t)nparts;
    int32_t *buf = wedge_buf + (int64_t)blockIdx.x * kWedgeCap;
    em.cached = 0;
    em.count = 0;
    em.hsum = 0;
    for (;;) {
        if (tid == 0) s_task = atomicAdd(cursor, 1u);
        __syncthreads();
        const uint64_t t = s_task;
        __syncthreads();
        if (t >= ntasks) break;
        const int32_t x = list[t / nparts];
        const int32_t part = (int32_t)(t % nparts);
        const int32_t z0 = part * kPartZ;
        const int32_t s = off[x], dx = off[x + 1] - s;
        for (int i = tid; i <= kPartZ; i += kBlock) cnt[i] = 0;
        __syncthreads();
        // wedges of this task restricted to z in [za, zb); pass 0 counts,
        // pass 1 places y into buf by z.
        auto walk = [&](int32_t za, int32_t zb, int pass) {
            for (int32_t c0 = 0; c0 < dx; c0 += kYChunk) {
                const int32_t i = c0 + tid;
                int32_t len = 0, start = 0, y = 0;
                if (i < dx) {
                    y = adj[s + i];
                    const int32_t dy = deg[y];
                    if (rank_less(dy, y, dx, x)) {
                        const int32_t *nyl = adj + off[y];
                        const int32_t lo = lower_bound_i32(nyl, dy, za);
                        const int32_t hi = lo + lower_bound_i32(nyl + lo, dy - lo, zb);
                        start = off[y] + lo;
                        len = hi - lo;
                    }
                }
                const int32_t inc = wave_incl_scan(len);
                if (lane == 63) s_sum[wid] = inc;
                __syncthreads();
                int32_t before = 0, total = 0;
                for (int q = 0; q < kWPB; q++) {
                    if (q < wid) before += s_sum[q];
                    total += s_sum[q];
                }
                s_pre[tid + 1] = before + inc;
                s_start[tid] = start;
                if (tid == 0) s_pre[0] = 0;
                __syncthreads();
                for (int32_t q = tid; q < total; q += kBlock) {
                    const int32_t j = last_le_i32(s_pre, kYChunk + 1, q);
                    const int32_t z = adj[s_start[j] + (q - s_pre[j])];
                    if (rank_less(deg[z], z, dx, x)) {
                        const int32_t zi = z - z0;
                        if (pass == 0) {
                            atomicAdd(&cnt[zi], 1);
                        } else {
                            const int32_t yj = adj[s + c0 + j];
                            const int32_t pos = cnt[zi] - cnt[za - z0] + (int32_t)atomicAdd(&cur[zi], 1u);
                            buf[pos] = yj;
                        }
                    }
                }
                __syncthreads();
            }
        };
        walk(z0, z0 + kPartZ, 0);
        // exclusive prefix of the counts (in place, cnt[kPartZ] = total)
        {
            constexpr int PER = kPartZ / kBlock;
            int32_t v[PER], sum = 0;
            for (int q = 0; q < PER; q++) {
                v[q] = cnt[tid * PER + q];
                sum += v[q];
            }
            const int32_t inc = wave_incl_scan(sum);
            if (lane == 63) s_sum[wid] = inc;
            __syncthreads();
            int32_t run = inc - sum;
            for (int q = 0; q < wid; q++) run += s_sum[q];
            for (int q = 0; q < PER; q++) {
                cnt[tid * PER + q] = run;
                run += v[q];
            }
            if (tid == kBlock - 1) cnt[kPartZ] = run;
            __syncthreads();
        }
        int32_t za = 0;   // relative to z0
        while (za < kPartZ && cnt[za] < cnt[kPartZ]) {
            // largest zb with cnt[zb] - cnt[za] <= kWedgeCap (at least za + 1)
            int32_t lo = za + 1, hi = kPartZ;
            while (lo < hi) {
                const int32_t mid = (lo + hi + 1) >> 1;
                if (cnt[mid] - cnt[za] <= kWedgeCap) lo = mid; else hi = mid - 1;
            }
            const int32_t zb = lo;
            for (int i = tid; i < kPartZ; i += kBlock) cur[i] = 0u;
            __syncthreads();
            walk(z0 + za, z0 + zb, 1);
            // emit: waves take z values of [za, zb) in turn
            if (tid == 0) s_z = (uint32_t)za;
            __syncthreads();
            for (;;) {
                uint32_t zi = 0;
                if (lane == 0) zi = atomicAdd(&s_z, 1u);
                zi = __shfl(zi, 0, 64);
                if ((int32_t)zi >= zb) break;
                const int32_t o = cnt[zi] - cnt[za], c = cnt[zi + 1] - cnt[zi];
                const int64_t np = (int64_t)c * (c - 1) / 2;
                for (int64_t qb = 0; qb < np; qb += kWave) {
                    const int64_t q = qb + lane;
                    const bool active = q < np;
                    int32_t y1 = 0, y2 = 0;
                    if (active) {
                        // q -> (i, j), i < j, q = j (j - 1) / 2 + i
                        int64_t j = (int64_t)((1.0 + sqrt(1.0 + 8.0 * (double)q)) * 0.5);
                        while (j * (j - 1) / 2 > q) j--;
                        while ((j + 1) * j / 2 <= q) j++;
                        const int64_t i = q - j * (j - 1) / 2;
                        y1 = buf[o + i];
                        y2 = buf[o + j];
                    }
                    emit_c4(em, active, x, y1, z0 + (int32_t)zi, y2);
                }
            }
            __syncthreads();
            za = zb;
        }
        __syncthreads();
    }
    emitter_flush(em, result);
}

__global__ void k_finish(unsigned long long *result, const unsigned long long *slot_ctr,
                         uint64_t cap) {
    if (threadIdx.x == 0 && blockIdx.x == 0) result[1] = *slot_ctr < cap ? *slot_ctr : cap;
}

struct C4Ws {
    uint32_t *ctl;                 // [0] heavy cursor, [1] light count, [2] heavy count
    unsigned long long *slot;      // listing slot counter
    unsigned long long *sum;       // counting: 128-bit total
    int32_t *deg, *cls, *flag, *pos, *light, *heavy;
    int64_t *scan_tmp;
    int32_t *wedges;               // listing: per-workgroup wedge buffers
    int2 *seg;                     // counting: part table (null when too large)
    int32_t *adeg;                 // counting: degree of each arc's end
    uint64_t bytes;
};

// 16-bit counters when at most one vertex (the top-ranked one, never a
// cycle's z) has a degree above 65535
bool narrow_counts(const gpm_graph *g) { return g->n_deg_over_65535 <= 1; }

int32_t count_zpart(const gpm_graph *g) { return narrow_counts(g) ? 2 * kCountWords : kCountWords; }

int32_t count_parts(const gpm_graph *g) {
    const int32_t z = count_zpart(g);
    return (int32_t)(((int64_t)g->n + z - 1) / z);
}

bool seg_table(const gpm_graph *g) {
    const int32_t np = count_parts(g);
    return np <= kSegMaxParts && (uint64_t)np * (uint64_t)g->n * sizeof(int2) <= kSegMaxBytes;
}

C4Ws c4_layout(const gpm_graph *g, bool list, void *base) {
    C4Ws W{};
    Carve c(base, ~0ull);
    const uint64_t n1 = (uint64_t)g->n + 1;
    W.ctl = c.take<uint32_t>(16);
    W.slot = c.take<unsigned long long>(2);
    W.sum = c.take<unsigned long long>(2);
    W.deg = c.take<int32_t>(n1);
    W.cls = c.take<int32_t>(n1);
    W.flag = c.take<int32_t>(n1);
    W.pos = c.take<int32_t>(n1);
    W.light = c.take<int32_t>(n1);
    W.heavy = c.take<int32_t>(n1);
    W.scan_tmp = c.take<int64_t>(scan_tmp_words(n1));
    if (list) W.wedges = c.take<int32_t>((uint64_t)kListBlocks * kWedgeCap);
    if (!list) {
        W.adeg = c.take<int32_t>((uint64_t)std::max<int64_t>(2 * g->m, 1));
        if (seg_table(g)) W.seg = c.take<int2>((uint64_t)count_parts(g) * (uint64_t)g->n);
    }
    W.bytes = c.used;
    return W;
}

unsigned grid_for(int64_t items, int per_block, int cap_per_cu) {
    int64_t b = (items + per_block - 1) / per_block;
    int64_t cap = (int64_t)cu_count() * cap_per_cu;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

}  // namespace

gpm_status c4_workspace_bytes(const gpm_graph *g, bool list, uint64_t *bytes) {
    if (list && g->max_degree > kWedgeCap)
        return fail(GPM_UNSUPPORTED, "4-cycle listing needs every degree <= 2^18");
    *bytes = c4_layout(g, list, nullptr).bytes;
    return GPM_OK;
}

// Counting (list == false): adds the number of 4-cycles to out128 (two
// 64-bit words, zero on entry); with cs (four words, zero on entry) and
// tsym (triangles per arc of the symmetric CSR) also the cycle sums of
// CycleSums.  Listing: fills d_result {total, written, checksum} (zeroed
// here) and d_buf rows (x, y1, z, y2) in cycle order.
gpm_status c4_run(const gpm_graph *g, bool list, void *ws, uint64_t ws_bytes,
                  unsigned long long *out128, int32_t *d_buf, uint64_t cap,
                  unsigned long long *d_result, hipStream_t st,
                  const uint32_t *tsym, unsigned long long *cs) {
    if (list && cs) return fail(GPM_INVALID_ARGUMENT, "cycle sums are a counting mode");
    C4Ws W = c4_layout(g, list, ws);
    if (W.bytes > ws_bytes) return fail(GPM_OUT_OF_MEMORY, "workspace smaller than required");
    if (list && g->max_degree > kWedgeCap)
        return fail(GPM_UNSUPPORTED, "4-cycle listing needs every degree <= 2^18");
    const int32_t n = g->n;
    GPM_HIP(fill_u32(W.ctl, 0, 16, st));
    GPM_HIP(fill_u32(W.slot, 0, 4, st));
    if (list) GPM_HIP(fill_u32(d_result, 0, 6, st));
    hipLaunchKernelGGL(k_degrees, dim3(grid_for(n, 256, 8)), dim3(256), 0, st, g->off, n, W.deg);
    hipLaunchKernelGGL(k_c4_work, dim3(grid_for(n, kWPB, 16)), dim3(kBlock), 0, st, g->off,
                       g->adj, W.deg, n, W.cls);
    GPM_LAUNCH_CHECK("k_c4_work");
    int32_t *cnt_light = (int32_t *)(W.ctl + 1), *cnt_heavy = (int32_t *)(W.ctl + 2);
    for (int cls = C4_LIGHT; cls <= C4_HEAVY; cls++) {
        int32_t *lst = cls == C4_LIGHT ? W.light : W.heavy;
        hipLaunchKernelGGL(k_flag_eq, dim3(grid_for(n, 256, 8)), dim3(256), 0, st, W.cls, n, cls,
                           W.flag);
        GPM_HIP(exclusive_scan_i32(W.flag, W.pos, (uint64_t)n, W.scan_tmp, st));
        hipLaunchKernelGGL(k_compact_eq, dim3(grid_for(n, 256, 8)), dim3(256), 0, st, W.cls,
                           W.pos, n, cls, lst);
        GPM_HIP(hipMemcpyAsync(cls == C4_LIGHT ? cnt_light : cnt_heavy, W.pos + n, 4,
                               hipMemcpyDeviceToDevice, st));
    }
    GPM_LAUNCH_CHECK("c4 classes");
    const int32_t nparts = (n + kPartZ - 1) / kPartZ;
    if (!list) {
        const int32_t cparts = count_parts(g);
        hipLaunchKernelGGL(k_arc_deg, dim3(grid_for(2 * g->m, 256, 16)), dim3(256), 0, st, g->adj,
                           W.deg, 2 * g->m, W.adeg);
        if (W.seg)
            hipLaunchKernelGGL(k_c4_seg, dim3(grid_for(n, kWPB, 8)), dim3(kBlock), 0, st, g->off,
                               g->adj, n, cparts, count_zpart(g), W.seg);
        GPM_LAUNCH_CHECK("k_c4_seg");
        if (cs) {
            Span sp("k_c4_heavy<sums>", st);
            hipLaunchKernelGGL(k_c4_heavy<true>, dim3((unsigned)cu_count()), dim3(kHeavyNT), 0, st,
                               g->off, g->adj, W.adeg, W.heavy, cnt_heavy, n, cparts,
                               narrow_counts(g) ? 1 : 0, W.seg, W.ctl + 0, out128, tsym, cs);
        } else {
            Span sp("k_c4_heavy", st);
            hipLaunchKernelGGL(k_c4_heavy<false>, dim3((unsigned)cu_count()), dim3(kHeavyNT), 0, st,
                               g->off, g->adj, W.adeg, W.heavy, cnt_heavy, n, cparts,
                               narrow_counts(g) ? 1 : 0, W.seg, W.ctl + 0, out128, nullptr,
                               nullptr);
        }
        GPM_LAUNCH_CHECK("k_c4_heavy");
        if (cs) {
            Span sp("k_c4_light<sums>", st);
            hipLaunchKernelGGL(k_c4_light<true>, dim3((unsigned)persistent_blocks(kWPB, 4)),
                               dim3(kBlock), 0, st, g->off, g->adj, W.deg, W.adeg, W.light,
                               cnt_light, out128, tsym, cs);
        } else {
            Span sp("k_c4_light", st);
            hipLaunchKernelGGL(k_c4_light<false>, dim3((unsigned)persistent_blocks(kWPB, 4)),
                               dim3(kBlock), 0, st, g->off, g->adj, W.deg, W.adeg, W.light,
                               cnt_light, out128, nullptr, nullptr);
        }
        GPM_LAUNCH_CHECK("k_c4_light");
        return GPM_OK;
    }
    Emitter em{W.slot, d_buf, d_buf ? cap : 0, 0, 0, 0};
    {
        Span sp("k_c4_heavy_list", st);
        hipLaunchKernelGGL(k_c4_heavy_list, dim3(kListBlocks), dim3(kBlock), 0, st, g->off, g->adj,
                           W.deg, W.heavy, cnt_heavy, nparts, W.ctl + 0, W.wedges, em, d_result);
    }
    GPM_LAUNCH_CHECK("k_c4_heavy_list");
    {
        Span sp("k_c4_light_list", st);
        hipLaunchKernelGGL(k_c4_light_list, dim3((unsigned)persistent_blocks(kWPB, 4)), dim3(kBlock),
                           0, st, g->off, g->adj, W.deg, W.light, cnt_light, em, d_result);
    }
    GPM_LAUNCH_CHECK("k_c4_light_list");
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(64), 0, st, d_result, W.slot, d_buf ? cap : 0);
    GPM_LAUNCH_CHECK("k_finish");
    return GPM_OK;
}

}  // namespace gpm
