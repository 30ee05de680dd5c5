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
// Counting runs on a copy of the graph relabelled by rank (below), where an
// apex's wedges are row prefixes, and sums C(c(x, z), 2) over the ends:
//   light apex (wedge work <= kLightW): one wave, LDS hash of the ends, each
//   new wedge to z adding the number of earlier ones;
//   medium apex (<= kMedW): one workgroup, a larger LDS hash;
//   heavy apex: tasks (x, part p) for z in the part's rank range, dense LDS
//   counters over the range, summed as they are cleared; each N(y) is
//   entered at the part through a part-major table of per-vertex segments,
//   or by binary search when the table would be too large.
// Listing (in vertex ids) groups each apex's wedges by z and emits every
// pair of middles: light apexes per wave, heavy ones per (apex, id part).
#include "gpm_internal.h"

#include <algorithm>

namespace gpm {

uint64_t row_sort_bytes(int32_t n);
gpm_status sort_rows(const int32_t *off, int32_t *adj, int32_t n, void *area, hipStream_t st);

namespace {

typedef unsigned __int128 u128;

constexpr int kBlock = 256;
constexpr int kWPB = kBlock / kWave;
constexpr int kLightW = 512;         // wedge work of a light apex
constexpr int kMedW = 8192;          // counting: wedge work of a medium apex (hashed task)
constexpr int kHashSlots = 1024;     // per-wave LDS hash (load <= 1/2)
constexpr int kPartZ = 8192;         // z-range per heavy task (LDS counters)
constexpr int kYChunk = kBlock;      // in-neighbours staged per round
constexpr int kListBlocks = 512;     // workgroups of the heavy listing kernel
constexpr int kWedgeCap = 1 << 18;   // per-workgroup wedge buffer (>= max degree)
constexpr int kListUnroll = 8;       // pairs per lane in flight when listing

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

enum C4Class : int { C4_NONE = 0, C4_LIGHT = 1, C4_HEAVY = 2, C4_MED = 3 };

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

// ------------------------------------------------- counting by rank ---
//
// Counting runs on a copy of the graph relabelled by rank in the degree
// order (c4_rank below): vertex r is the r-th in degree order, ties in any
// order (any total order gives each cycle one top vertex), and every row
// lists its neighbours' ranks ascending.  The wedges of apex x are then
// prefixes: its in-neighbours y < x are the entries of row x below x, and
// the ends z < x of a middle y the entries of row y below x, so no wedge is
// read only to fail a rank test and no end's degree is read (4 B per wedge
// instead of 8).  A z-part [z0, z1) of the counters is a range of ranks,
// hence one segment of every row.

// Per apex x: nin[x] = its in-neighbours (entries of row x below x) and
// its class by the exact wedge work, the sum over them of the entries of
// their rows below x (the position of x in row y): light up to kLightW,
// medium up to kMedW, heavy beyond.  The sum of their degrees bounds it: at
// most kLightW settles the class without the searches, and the exact sum
// stops once past kMedW.  A wave per apex.
__global__ void __launch_bounds__(kBlock) k_c4r_work(const int32_t *__restrict__ roff,
                                                     const int32_t *__restrict__ radj, int32_t n,
                                                     int32_t *nin, int32_t *cls) {
    const int lane = lane_id();
    const int64_t wave0 = (int64_t)blockIdx.x * kWPB + threadIdx.x / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * kWPB;
    for (int64_t r = wave0; r < n; r += nwaves) {
        const int32_t x = (int32_t)r, s = roff[x], dx = roff[x + 1] - s;
        const int32_t k = lower_bound_i32(radj + s, dx, x);
        int64_t b = 0;
        for (int32_t i = lane; i < k && b <= kLightW; i += kWave) {
            const int32_t y = radj[s + i];
            b += roff[y + 1] - roff[y];
        }
        b = wave_sum(b);
        int64_t w = 0;
        if (b > kLightW)
            for (int32_t i0 = 0; i0 < k && w <= kMedW; i0 += kWave) {
                int64_t c = 0;
                if (i0 + lane < k) {
                    const int32_t y = radj[s + i0 + lane], sy = roff[y];
                    c = lower_bound_i32(radj + sy, roff[y + 1] - sy, x);
                }
                w += wave_sum(c);
            }
        if (lane == 0) {
            nin[x] = k;
            cls[x] = k < 2 ? C4_NONE
                     : b <= kLightW || w <= kLightW ? C4_LIGHT
                     : w <= kMedW ? C4_MED : C4_HEAVY;
        }
    }
}

// Light apexes: one wave each, LDS hash z -> count, wedge by wedge.  The
// staged middles are the in-neighbours with an end below x: base[j] = the
// start of y_j's row, pre[j + 1] = prefix of their end counts (the wedge
// work, at most kLightW), and with CS dy[j] = d(y_j), arcs[j] = the arc
// x -> y_j.  With CS, a second walk over the apex's wedges adds the cycle
// sums.
template <bool CS>
__global__ void __launch_bounds__(kBlock) k_c4r_light(const int32_t *__restrict__ roff,
                                                      const int32_t *__restrict__ radj,
                                                      const int32_t *__restrict__ nin,
                                                      const int32_t *__restrict__ list,
                                                      const int32_t *__restrict__ count_p,
                                                      unsigned long long *out,
                                                      const uint32_t *__restrict__ rtsym,
                                                      unsigned long long *cs) {
    __shared__ int32_t s_key[kWPB][kHashSlots];
    __shared__ uint32_t s_cnt[kWPB][kHashSlots];
    __shared__ int32_t s_pre[kWPB][kLightW + 1];
    __shared__ int32_t s_base[kWPB][kLightW];
    __shared__ int32_t s_arc[CS ? kWPB : 1][CS ? kLightW : 1];
    __shared__ int32_t s_dy[CS ? kWPB : 1][CS ? kLightW : 1];
    const int lane = lane_id(), wib = threadIdx.x / kWave;
    int32_t *key = s_key[wib], *pre = s_pre[wib], *base = s_base[wib];
    uint32_t *cnt = s_cnt[wib];
    const int32_t count = *count_p;
    const int64_t wave0 = (int64_t)blockIdx.x * kWPB + wib;
    const int64_t nwaves = (int64_t)gridDim.x * kWPB;
    for (int i = lane; i < kHashSlots; i += kWave) { key[i] = -1; cnt[i] = 0; }
    uint64_t acc = 0;
    CycleSums sums;
    for (int64_t r = wave0; r < count; r += nwaves) {
        const int32_t x = list[r], s = roff[x], k = nin[x];
        // stage the middles with at least one end below x
        int32_t ny = 0, W = 0;
        for (int32_t i0 = 0; i0 < k; i0 += kWave) {
            const int32_t i = i0 + lane;
            int32_t y = 0, sy = 0, wy = 0;
            if (i < k) {
                y = radj[s + i];
                sy = roff[y];
                wy = lower_bound_i32(radj + sy, roff[y + 1] - sy, x);
            }
            const bool in = wy > 0;
            const uint64_t mask = __ballot(in);
            const int32_t p = ny + lanes_below(mask);
            const int32_t inc = wave_incl_scan(wy);
            if (in) {
                base[p] = sy;
                pre[p + 1] = W + inc;
                if (CS) {
                    s_arc[wib][p] = s + i;
                    s_dy[wib][p] = roff[y + 1] - sy;
                }
            }
            W += __shfl(inc, 63, 64);
            ny += __popcll(mask);
        }
        if (lane == 0) pre[0] = 0;
        wave_sync();
        for (int32_t qb = 0; qb < W; qb += kWave) {
            const int32_t q = qb + lane;
            if (q < W) {
                const int32_t j = last_le_i32(pre, ny + 1, q);
                const int32_t z = radj[base[j] + (q - pre[j])];
                uint32_t h = hash_slot(z);
                for (;;) {
                    int32_t kk = key[h];
                    if (kk == -1) {
                        kk = atomicCAS(&key[h], -1, z);
                        if (kk == -1) kk = z;
                    }
                    if (kk == z) {
                        acc += atomicAdd(&cnt[h], 1u);
                        break;
                    }
                    h = (h + 1) & (kHashSlots - 1);
                }
            }
        }
        wave_sync();
        if (CS) {
            const uint32_t dx = (uint32_t)(roff[x + 1] - s);
            for (int32_t qb = 0; qb < W; qb += kWave) {
                const int32_t q = qb + lane;
                if (q < W) {
                    const int32_t j = last_le_i32(pre, ny + 1, q);
                    const int32_t e = base[j] + (q - pre[j]);
                    const int32_t z = radj[e];
                    uint32_t h = hash_slot(z);
                    while (key[h] != z) h = (h + 1) & (kHashSlots - 1);
                    sums.add(cnt[h], dx, (uint32_t)s_dy[wib][j], (uint32_t)(roff[z + 1] - roff[z]),
                             rtsym[s_arc[wib][j]], rtsym[e]);
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
// tasks running together share one part's table row.  The block keeps a
// dense LDS counter per z of the part; for each in-neighbour y of x it
// takes the segment of row y inside the part (from the part table, else by
// binary search), cut at x in the part that holds x (parts above x have no
// ends and are skipped), and the block walks the concatenated segments, one
// wedge per lane, adding one to the counter of its end z; reading the
// counters back as it clears them for the next task, it adds C(c, 2) for
// each.  A counter c(x, z) never exceeds deg(z), and z, ranked
// below x, is never the top-ranked vertex, so when at most one vertex has a
// degree above 65535 the counters are 16 bits, two to a word, and a part
// spans 65536 ranks instead of 32768: half the tasks, segments twice as
// long.  With CS, a second walk over the task's wedges, once its counters
// are complete, adds the cycle sums (CycleSums above).
// A medium apex (wedge work up to kMedW) is one task over every z < x
// instead of one per part: the counter words hold an open-addressing hash
// z + 1 -> count (keys in the first half, counts in the second; all zero is
// empty), so the part table, the cut and most of the per-task set-up go.
constexpr int kCountWords = 32768;   // LDS counter words of a counting task (128 KiB)
constexpr int kMedSlots = kCountWords / 2;
static_assert(kMedSlots >= 2 * kMedW, "medium hash load at most 1/2");

__device__ __forceinline__ uint32_t med_slot(int32_t z) {
    return ((uint32_t)z * 0x9E3779B1u) >> 18;   // 14 bits -> kMedSlots
}
static_assert(kMedSlots == 1 << 14, "med_slot yields 14 bits");
constexpr int kHeavyNT = 1024;
constexpr int kUnroll = 8;           // wedges in flight per lane
constexpr int kSegMaxParts = 256;    // part table only for graphs of at most 256 parts
constexpr uint64_t kSegMaxBytes = 2ull << 30;

// Part table: seg[p * n + y] = {first entry of row y with value >= p * zpart,
// number of entries of row y with value in part p}.  A thread per row finds
// each part's first entry by a binary search from the previous one, so the
// threads of a wave write consecutive entries of each part's table row.
__global__ void __launch_bounds__(kBlock) k_c4_seg(const int32_t *__restrict__ off,
                                                   const int32_t *__restrict__ adj, int32_t n,
                                                   int32_t nparts, int32_t zpart, int2 *seg) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t y = (int64_t)blockIdx.x * kBlock + threadIdx.x; y < n; y += stride) {
        const int32_t s = off[y], d = off[y + 1] - s;
        int32_t lo = 0;
        for (int32_t q = 0; q < nparts; q++) {
            const int64_t zend = (int64_t)(q + 1) * zpart;
            const int32_t hi = zend >= n ? d
                                          : lo + lower_bound_i32(adj + s + lo, d - lo, (int32_t)zend);
            seg[(int64_t)q * n + y] = make_int2(s + lo, hi - lo);
            lo = hi;
        }
    }
}

// C(c, 2) of one counter word: two 16-bit counters when narrow, else one.
__device__ __forceinline__ uint64_t pairs_of(uint32_t w, bool narrow) {
    const uint64_t a = narrow ? (w & 0xffffu) : w, b = narrow ? (w >> 16) : 0u;
    return (a * (a - 1) + b * (b - 1)) / 2;   // 0 for a zero counter (unsigned wrap times 0)
}

// Last j in [lo, hi) with pre[j] <= q, given pre[lo] <= q.
__device__ __forceinline__ int32_t seg_of(const int32_t *pre, int32_t lo, int32_t hi, int32_t q) {
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (pre[mid] <= q) lo = mid; else hi = mid;
    }
    return lo;
}

template <bool CS>
__global__ void __launch_bounds__(kHeavyNT) k_c4r_heavy(const int32_t *__restrict__ roff,
                                                        const int32_t *__restrict__ radj,
                                                        const int32_t *__restrict__ nin,
                                                        const int32_t *__restrict__ list,
                                                        const int32_t *__restrict__ count_p,
                                                        const int32_t *__restrict__ med,
                                                        const int32_t *__restrict__ count_med,
                                                        int32_t n, int32_t nparts, int32_t narrow,
                                                        const int2 *__restrict__ seg,
                                                        uint32_t *cursor, unsigned long long *out,
                                                        const uint32_t *__restrict__ rtsym,
                                                        unsigned long long *cs) {
    constexpr int NW = kHeavyNT / kWave;
    __shared__ __align__(16) uint32_t cnt[kCountWords];
    __shared__ int32_t s_pre[kHeavyNT + 1];
    __shared__ int32_t s_off[kHeavyNT];    // segment start minus its pair prefix
    __shared__ int32_t s_sum[NW];
    __shared__ uint32_t s_dy[CS ? kHeavyNT : 1];    // d(y) of each segment
    __shared__ uint32_t s_txy[CS ? kHeavyNT : 1];   // triangles on the arc x -> y
    __shared__ uint32_t s_task;
    const int tid = threadIdx.x, lane = lane_id(), wid = tid / kWave;
    const int32_t nheavy = *count_p, nmed = *count_med;
    const uint64_t nparted = (uint64_t)nheavy * (uint64_t)nparts;
    const uint64_t ntasks = nparted + (uint64_t)nmed;
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
        // the heavy apexes' parts first, then the medium apexes; parts from
        // the top down and, within a part, apexes by descending rank: the top
        // part holds most of the hubs' ends, so the largest tasks start
        // first, and a part's tail is apexes below it, which have no work
        // there
        const bool hashed = t >= nparted;
        int32_t row = 0, x, z0 = 0, z1 = 0;   // row: the part (of the part table)
        if (hashed) {
            x = med[nmed - 1 - (int32_t)(t - nparted)];
        } else {
            row = nparts - 1 - (int32_t)(t / (uint64_t)nheavy);
            x = list[nheavy - 1 - (int32_t)(t % (uint64_t)nheavy)];
            z0 = row * zpart;
            z1 = (int32_t)min<int64_t>((int64_t)z0 + zpart, n);
            if (z0 >= x) continue;   // no end of x in this part (the same for the block)
        }
        const bool cut = z1 > x;   // the range holds x: stop the segments at x
        if (cut) z1 = x;
        const int32_t s = roff[x], k = nin[x];
        const uint32_t dx = (uint32_t)(roff[x + 1] - s);
        for (int pass = 0; pass < (CS ? 2 : 1); pass++)
        for (int32_t c0 = 0; c0 < k; c0 += kHeavyNT) {
            const int32_t i = c0 + tid;
            int32_t len[1] = {0}, start = 0;
            if (i < k) {
                const int32_t y = radj[s + i];
                const int32_t sy = roff[y], dy = roff[y + 1] - sy;
                if (hashed) {
                    start = sy;
                    len[0] = lower_bound_i32(radj + sy, dy, x);
                } else if (seg) {
                    const int2 sg = seg[(int64_t)row * n + y];
                    start = sg.x;
                    len[0] = cut ? lower_bound_i32(radj + sg.x, sg.y, x) : sg.y;
                } else {
                    const int32_t lo = lower_bound_i32(radj + sy, dy, z0);
                    const int32_t hi = lo + lower_bound_i32(radj + sy + lo, dy - lo, z1);
                    start = sy + lo;
                    len[0] = hi - lo;
                }
                if (CS) {
                    s_dy[tid] = (uint32_t)dy;
                    s_txy[tid] = rtsym[s + i];
                }
            }
            block_prefix<kHeavyNT, 1>(len, kHeavyNT, s_pre, s_sum);   // ends with a barrier
            s_off[tid] = start - s_pre[tid];
            __syncthreads();
            const int32_t total = s_pre[kHeavyNT];
            // each wave walks a contiguous range of the chunk's wedges; a
            // lane finds each wedge's segment by a branchless search over
            // the segments the wave's range spans, its kUnroll searches in
            // step, then loads the kUnroll ends together and counts them
            const int32_t per_wave = ((total + NW - 1) / NW + kWave - 1) / kWave * kWave;
            const int32_t qa = min(total, wid * per_wave);
            const int32_t qz = min(total, qa + per_wave);
            if (qa < qz) {
                int32_t ja = seg_of(s_pre, 0, kHeavyNT, qa);
                const int32_t jz = seg_of(s_pre, ja, kHeavyNT, qz - 1) + 1;
                for (int32_t qb = qa; qb < qz; qb += kWave * kUnroll) {
                    int32_t jj[kUnroll], z[kUnroll], e[kUnroll];
#pragma unroll
                    for (int u = 0; u < kUnroll; u++) jj[u] = ja;
                    for (int32_t len = jz - ja; len > 1;) {
                        const int32_t half = len >> 1;
#pragma unroll
                        for (int u = 0; u < kUnroll; u++)
                            if (s_pre[jj[u] + half] <= qb + u * kWave + lane) jj[u] += half;
                        len -= half;
                    }
#pragma unroll
                    for (int u = 0; u < kUnroll; u++) e[u] = s_off[jj[u]] + qb + u * kWave + lane;
#pragma unroll
                    for (int u = 0; u < kUnroll; u++)
                        z[u] = qb + u * kWave + lane < qz ? radj[e[u]] : z0;
#pragma unroll
                    for (int u = 0; u < kUnroll; u++) {
                        if (qb + u * kWave + lane >= qz) continue;
                        if (hashed) {
                            const uint32_t key = (uint32_t)z[u] + 1u;
                            uint32_t h = med_slot(z[u]);
                            if (pass == 0) {
                                for (;;) {
                                    uint32_t kk = cnt[h];
                                    if (kk == 0u) {
                                        kk = atomicCAS(&cnt[h], 0u, key);
                                        if (kk == 0u) kk = key;
                                    }
                                    if (kk == key) break;
                                    h = (h + 1) & (kMedSlots - 1);
                                }
                                atomicAdd(&cnt[kMedSlots + h], 1u);
                            } else {
                                while (cnt[h] != key) h = (h + 1) & (kMedSlots - 1);
                                sums.add(cnt[kMedSlots + h], dx, s_dy[jj[u]],
                                         (uint32_t)(roff[z[u] + 1] - roff[z[u]]), s_txy[jj[u]],
                                         rtsym[e[u]]);
                            }
                            continue;
                        }
                        const uint32_t zz = (uint32_t)(z[u] - z0);
                        const uint32_t sh = narrow ? (zz & 1u) * 16u : 0u;
                        uint32_t *cw = narrow ? &cnt[zz >> 1] : &cnt[zz];
                        if (pass == 0) {
                            atomicAdd(cw, narrow ? 1u << sh : 1u);
                        } else {
                            const uint32_t c = narrow ? (*cw >> sh) & 0xffffu : *cw;
                            sums.add(c, dx, s_dy[jj[u]],
                                     (uint32_t)(roff[z[u] + 1] - roff[z[u]]), s_txy[jj[u]],
                                     rtsym[e[u]]);
                        }
                    }
                    // the next step's wedges start at or after the last one here
                    ja = __shfl(jj[kUnroll - 1], kWave - 1, kWave);
                }
            }
            __syncthreads();
        }
        // C(c, 2) of every counter (the keys of a hashed task count no
        // pairs), read as the counters are cleared for the next task
        {
            uint4 *c4 = reinterpret_cast<uint4 *>(cnt);
            const int i0 = hashed ? kMedSlots / 4 : 0;
            for (int i = i0 + tid; i < kCountWords / 4; i += kHeavyNT) {
                const uint4 v = c4[i];
                acc += pairs_of(v.x, narrow && !hashed) + pairs_of(v.y, narrow && !hashed) +
                       pairs_of(v.z, narrow && !hashed) + pairs_of(v.w, narrow && !hashed);
            }
            for (int i = tid; i < kCountWords / 4; i += kHeavyNT) c4[i] = make_uint4(0, 0, 0, 0);
        }
        __syncthreads();
    }
    acc = wave_sum(acc);
    if (lane == 0 && acc) atomic_add_u128(out, (u128)acc);
    if (CS) sums.flush(cs);
}

// ------------------------------------------------------ relabelling ---
// Ranks in the degree order, ties in any order: rank[v] = (vertices of
// smaller degree) + a slot among v's degree.  A workgroup groups its
// kGroupV vertices by degree in an LDS hash (at most kGroupV keys in twice
// as many slots) so that each distinct degree costs one global atomic per
// workgroup, not one per vertex (a few small degrees hold most vertices).
constexpr int kGroupPer = 8;                  // vertices per thread
constexpr int kGroupV = kBlock * kGroupPer;   // vertices per workgroup
constexpr int kGroupSlots = 2 * kGroupV;

__device__ __forceinline__ uint32_t group_slot(int32_t d) {
    return ((uint32_t)d * 0x9E3779B1u) >> 20;   // 12 bits -> kGroupSlots
}
static_assert(kGroupSlots == 1 << 12, "group_slot yields 12 bits");

// ASSIGN = false: dcnt[d] += vertices of degree d.  ASSIGN = true: ranks
// from dstart (exclusive prefix of dcnt) and the per-degree cursors dcur;
// perm[rank] = v, rdeg[rank] = d.
template <bool ASSIGN>
__global__ void __launch_bounds__(kBlock) k_rank_group(const int32_t *__restrict__ off, int32_t n,
                                                       int32_t *dcnt, const int32_t *dstart,
                                                       int32_t *dcur, int32_t *rank, int32_t *perm,
                                                       int32_t *rdeg) {
    __shared__ int32_t key[kGroupSlots];
    __shared__ int32_t num[kGroupSlots];
    for (int i = threadIdx.x; i < kGroupSlots; i += kBlock) {
        key[i] = -1;
        num[i] = 0;
    }
    __syncthreads();
    const int64_t v0 = (int64_t)blockIdx.x * kGroupV + threadIdx.x;
    int32_t d[kGroupPer], slot[kGroupPer], local[kGroupPer];
#pragma unroll
    for (int u = 0; u < kGroupPer; u++) {
        const int64_t v = v0 + (int64_t)u * kBlock;
        d[u] = v < n ? off[v + 1] - off[v] : -1;
    }
#pragma unroll
    for (int u = 0; u < kGroupPer; u++) {
        slot[u] = 0;
        local[u] = 0;
        if (d[u] < 0) continue;
        uint32_t h = group_slot(d[u]);
        for (;;) {
            int32_t k = key[h];
            if (k == -1) {
                k = atomicCAS(&key[h], -1, d[u]);
                if (k == -1) k = d[u];
            }
            if (k == d[u]) break;
            h = (h + 1) & (kGroupSlots - 1);
        }
        slot[u] = (int32_t)h;
        local[u] = atomicAdd(&num[h], 1);
    }
    __syncthreads();
    // num[] becomes the slot's first rank (ASSIGN)
    for (int i = threadIdx.x; i < kGroupSlots; i += kBlock)
        if (key[i] != -1) {
            if (ASSIGN) num[i] = dstart[key[i]] + atomicAdd(&dcur[key[i]], num[i]);
            else atomicAdd(&dcnt[key[i]], num[i]);
        }
    if (!ASSIGN) return;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kGroupPer; u++) {
        if (d[u] < 0) continue;
        const int64_t v = v0 + (int64_t)u * kBlock;
        const int32_t r = num[slot[u]] + local[u];
        rank[v] = r;
        perm[r] = (int32_t)v;
        rdeg[r] = d[u];
    }
}

// Row rank[v] of the relabelled graph: the ranks of v's neighbours (sorted
// afterwards).  A wave takes 4 consecutive vertices, a 16-lane group each;
// rows longer than kRowGroupMax are then done by the whole wave, kRowUnroll
// entries per lane in flight (a hub's row would otherwise be a long chain
// of dependent gathers).
constexpr int kRowGroup = 16;
constexpr int kRowGroupMax = 64;
constexpr int kRowUnroll = 8;

__global__ void __launch_bounds__(kBlock) k_rank_rows(const int32_t *__restrict__ off,
                                                      const int32_t *__restrict__ adj, int32_t n,
                                                      const int32_t *__restrict__ rank,
                                                      const int32_t *__restrict__ roff,
                                                      int32_t *radj) {
    constexpr int kPer = kWave / kRowGroup;
    const int lane = lane_id(), gl = lane % kRowGroup, grp = lane / kRowGroup;
    const int64_t wave0 = (int64_t)blockIdx.x * kWPB + threadIdx.x / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * kWPB;
    for (int64_t v0 = wave0 * kPer; v0 < n; v0 += nwaves * kPer) {
        const int64_t v = v0 + grp;
        int32_t s = 0, d = 0, r = 0;
        if (v < n) {
            s = off[v];
            d = off[v + 1] - s;
            r = roff[rank[v]];
        }
        if (d <= kRowGroupMax)
            for (int32_t i = gl; i < d; i += kRowGroup) radj[r + i] = rank[adj[s + i]];
        uint64_t longs = __ballot(d > kRowGroupMax && gl == 0);
        while (longs) {
            const int src = __builtin_ctzll(longs);
            longs &= longs - 1ull;
            const int32_t ls = __shfl(s, src, kWave), ld = __shfl(d, src, kWave);
            const int32_t lr = __shfl(r, src, kWave);
            for (int32_t i0 = 0; i0 < ld; i0 += kWave * kRowUnroll) {
                int32_t w[kRowUnroll];
#pragma unroll
                for (int u = 0; u < kRowUnroll; u++) {
                    const int32_t i = i0 + u * kWave + lane;
                    w[u] = i < ld ? adj[ls + i] : 0;
                }
#pragma unroll
                for (int u = 0; u < kRowUnroll; u++) {
                    const int32_t i = i0 + u * kWave + lane;
                    if (i < ld) radj[lr + i] = rank[w[u]];
                }
            }
        }
    }
}

// Triangle counts per arc of the relabelled graph (for the cycle sums):
// arc (r -> t) is arc (perm[r] -> perm[t]) of the symmetric CSR, found by
// binary search in the row of perm[r].
__global__ void __launch_bounds__(kBlock) k_rank_tsym(const int32_t *__restrict__ off,
                                                      const int32_t *__restrict__ adj, int32_t n,
                                                      const int32_t *__restrict__ perm,
                                                      const int32_t *__restrict__ roff,
                                                      const int32_t *__restrict__ radj,
                                                      const uint32_t *__restrict__ tsym,
                                                      uint32_t *rtsym) {
    const int lane = lane_id();
    const int64_t wave0 = (int64_t)blockIdx.x * kWPB + threadIdx.x / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * kWPB;
    for (int64_t r = wave0; r < n; r += nwaves) {
        const int32_t u = perm[r], su = off[u], du = off[u + 1] - su;
        const int32_t s = roff[r], d = roff[r + 1] - s;
        for (int32_t i = lane; i < d; i += kWave) {
            const int32_t w = perm[radj[s + i]];
            rtsym[s + i] = tsym[su + lower_bound_i32(adj + su, du, w)];
        }
    }
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
    __shared__ int64_t s_pp[kWPB][kWave];   // per wave: first pair of each of its 64 z
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
            // emit: waves take 64 consecutive z of [za, zb) at a time and
            // share out the pairs of middles of all of them, one per lane
            // (most groups hold one or two pairs, so a wave per z would
            // leave most lanes idle)
            if (tid == 0) s_z = (uint32_t)za;
            __syncthreads();
            int64_t *pp = s_pp[wid];
            for (;;) {
                uint32_t z1 = 0;
                if (lane == 0) z1 = atomicAdd(&s_z, (uint32_t)kWave);
                z1 = __shfl(z1, 0, 64);
                if ((int32_t)z1 >= zb) break;
                const int32_t zl = (int32_t)z1 + lane;
                const int32_t cl = zl < zb ? cnt[zl + 1] - cnt[zl] : 0;
                const int64_t npl = (int64_t)cl * (cl - 1) / 2;
                const int64_t incl = wave_incl_scan(npl);
                pp[lane] = incl - npl;   // first pair of this lane's z
                const int64_t total = __shfl(incl, kWave - 1, 64);
                wave_sync();
                // each lane takes kListUnroll consecutive pairs per step:
                // it decodes the first and steps through the rest (a new z's
                // pairs start at (0, 1)), and their middles' loads go out
                // together before any is hashed
                for (int64_t qb = 0; qb < total; qb += kWave * kListUnroll) {
                    const int64_t q0 = qb + (int64_t)lane * kListUnroll;
                    int32_t y1[kListUnroll], y2[kListUnroll], zz[kListUnroll];
                    int32_t l = 0, o = 0, c = 0, i = 0, j = 0;
                    // the lane (z) holding pair q: last l with pp[l] <= q
                    auto find = [&](int64_t q) {
                        l = 0;
#pragma unroll
                        for (int h = kWave / 2; h > 0; h >>= 1)
                            if (pp[l + h] <= q) l += h;
                        o = cnt[(int32_t)z1 + l] - cnt[za];
                        c = cnt[(int32_t)z1 + l + 1] - cnt[(int32_t)z1 + l];
                    };
                    if (q0 < total) {
                        find(q0);
                        // r -> (i, j), i < j, r = j (j - 1) / 2 + i; the
                        // single-precision root is off by at most one here
                        const int64_t r = q0 - pp[l];
                        int64_t jj = (int64_t)((1.0f + sqrtf(1.0f + 8.0f * (float)r)) * 0.5f);
                        while (jj * (jj - 1) / 2 > r) jj--;
                        while ((jj + 1) * jj / 2 <= r) jj++;
                        j = (int32_t)jj;
                        i = (int32_t)(r - jj * (jj - 1) / 2);
                    }
#pragma unroll
                    for (int u = 0; u < kListUnroll; u++) {
                        const int64_t q = q0 + u;
                        y1[u] = y2[u] = zz[u] = 0;
                        if (q < total) {
                            if (u > 0 && ++i == j) {
                                i = 0;
                                if (++j == c) {   // this z's pairs are done
                                    find(q);
                                    j = 1;
                                }
                            }
                            zz[u] = (int32_t)z1 + l;
                            y1[u] = buf[o + i];
                            y2[u] = buf[o + j];
                        }
                    }
#pragma unroll
                    for (int u = 0; u < kListUnroll; u++)
                        emit_c4(em, q0 + u < total, x, y1[u], z0 + zz[u], y2[u]);
                }
                wave_sync();
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
    uint32_t *ctl;                 // [0] heavy cursor; counts [1] light, [2] heavy, [3] medium
    unsigned long long *slot;      // listing slot counter
    unsigned long long *sum;       // counting: 128-bit total
    int32_t *deg, *cls, *flag, *pos, *light, *heavy, *med;
    int64_t *scan_tmp;
    int32_t *wedges;               // listing: per-workgroup wedge buffers
    int2 *seg;                     // counting: part table (null when too large)
    // counting: the graph relabelled by rank (see above) and its build
    int32_t *rank, *perm, *rdeg, *roff, *radj, *nin, *dcnt, *dstart, *dcur;
    uint32_t *rtsym;               // with cycle sums: triangles per relabelled arc
    void *sort_area;
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
        const uint64_t arcs = (uint64_t)std::max<int64_t>(2 * g->m, 1);
        W.med = c.take<int32_t>(n1);
        W.rank = c.take<int32_t>(n1);
        W.perm = c.take<int32_t>(n1);
        W.rdeg = c.take<int32_t>(n1);
        W.roff = c.take<int32_t>(n1);
        W.nin = c.take<int32_t>(n1);
        W.dcnt = c.take<int32_t>(n1);
        W.dstart = c.take<int32_t>(n1);
        W.dcur = c.take<int32_t>(n1);
        W.radj = c.take<int32_t>(arcs);
        W.rtsym = c.take<uint32_t>(arcs);
        W.sort_area = c.take<char>(row_sort_bytes(g->n));
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
    int32_t *cnt_light = (int32_t *)(W.ctl + 1), *cnt_heavy = (int32_t *)(W.ctl + 2);
    int32_t *cnt_med = (int32_t *)(W.ctl + 3);
    // the apex lists of each class (medium only when counting)
    auto split_classes = [&]() -> gpm_status {
        for (int cls = C4_LIGHT; cls <= (list ? C4_HEAVY : C4_MED); cls++) {
            int32_t *lst = cls == C4_LIGHT ? W.light : cls == C4_HEAVY ? W.heavy : W.med;
            int32_t *lcnt = (int32_t *)(W.ctl + cls);
            hipLaunchKernelGGL(k_flag_eq, dim3(grid_for(n, 256, 8)), dim3(256), 0, st, W.cls, n,
                               cls, W.flag);
            GPM_HIP(exclusive_scan_i32(W.flag, W.pos, (uint64_t)n, W.scan_tmp, st));
            hipLaunchKernelGGL(k_compact_eq, dim3(grid_for(n, 256, 8)), dim3(256), 0, st, W.cls,
                               W.pos, n, cls, lst);
            GPM_HIP(hipMemcpyAsync(lcnt, W.pos + n, 4, hipMemcpyDeviceToDevice, st));
        }
        GPM_LAUNCH_CHECK("c4 classes");
        return GPM_OK;
    };
    if (!list) {
        // the graph relabelled by rank in the degree order
        {
            Span sp("c4_rank", st);
            const uint64_t dn = (uint64_t)g->max_degree + 1;
            GPM_HIP(fill_u32(reinterpret_cast<uint32_t *>(W.dcnt), 0, dn, st));
            GPM_HIP(fill_u32(reinterpret_cast<uint32_t *>(W.dcur), 0, dn, st));
            const unsigned gb = (unsigned)std::max<int64_t>(1, ((int64_t)n + kGroupV - 1) / kGroupV);
            if (n > 0) {
                hipLaunchKernelGGL(k_rank_group<false>, dim3(gb), dim3(kBlock), 0, st, g->off, n,
                                   W.dcnt, nullptr, nullptr, nullptr, nullptr, nullptr);
                GPM_HIP(exclusive_scan_i32(W.dcnt, W.dstart, dn, W.scan_tmp, st));
                hipLaunchKernelGGL(k_rank_group<true>, dim3(gb), dim3(kBlock), 0, st, g->off, n,
                                   nullptr, W.dstart, W.dcur, W.rank, W.perm, W.rdeg);
            }
            GPM_LAUNCH_CHECK("k_rank_group");
            GPM_HIP(exclusive_scan_i32(W.rdeg, W.roff, (uint64_t)n, W.scan_tmp, st));
            hipLaunchKernelGGL(k_rank_rows, dim3(grid_for(n, kWPB * (kWave / kRowGroup), 16)),
                               dim3(kBlock), 0, st,
                               g->off, g->adj, n, W.rank, W.roff, W.radj);
            GPM_LAUNCH_CHECK("k_rank_rows");
            gpm_status src = sort_rows(W.roff, W.radj, n, W.sort_area, st);
            if (src) return src;
            if (cs) {
                hipLaunchKernelGGL(k_rank_tsym, dim3(grid_for(n, kWPB, 16)), dim3(kBlock), 0, st,
                                   g->off, g->adj, n, W.perm, W.roff, W.radj, tsym, W.rtsym);
                GPM_LAUNCH_CHECK("k_rank_tsym");
            }
        }
        hipLaunchKernelGGL(k_c4r_work, dim3(grid_for(n, kWPB, 16)), dim3(kBlock), 0, st, W.roff,
                           W.radj, n, W.nin, W.cls);
        GPM_LAUNCH_CHECK("k_c4r_work");
        gpm_status rc = split_classes();
        if (rc) return rc;
        const int32_t cparts = count_parts(g);
        if (W.seg)
            hipLaunchKernelGGL(k_c4_seg, dim3(grid_for(n, kBlock, 8)), dim3(kBlock), 0, st, W.roff,
                               W.radj, n, cparts, count_zpart(g), W.seg);
        GPM_LAUNCH_CHECK("k_c4_seg");
        const int narrow = narrow_counts(g) ? 1 : 0;
        if (cs) {
            Span sp("k_c4_heavy<sums>", st);
            hipLaunchKernelGGL(k_c4r_heavy<true>, dim3((unsigned)cu_count()), dim3(kHeavyNT), 0,
                               st, W.roff, W.radj, W.nin, W.heavy, cnt_heavy, W.med, cnt_med, n,
                               cparts, narrow, W.seg, W.ctl + 0, out128, W.rtsym, cs);
        } else {
            Span sp("k_c4_heavy", st);
            hipLaunchKernelGGL(k_c4r_heavy<false>, dim3((unsigned)cu_count()), dim3(kHeavyNT), 0,
                               st, W.roff, W.radj, W.nin, W.heavy, cnt_heavy, W.med, cnt_med, n,
                               cparts, narrow, W.seg, W.ctl + 0, out128, nullptr, nullptr);
        }
        GPM_LAUNCH_CHECK("k_c4_heavy");
        if (cs) {
            Span sp("k_c4_light<sums>", st);
            hipLaunchKernelGGL(k_c4r_light<true>, dim3((unsigned)persistent_blocks(kWPB, 4)),
                               dim3(kBlock), 0, st, W.roff, W.radj, W.nin, W.light, cnt_light,
                               out128, W.rtsym, cs);
        } else {
            Span sp("k_c4_light", st);
            hipLaunchKernelGGL(k_c4r_light<false>, dim3((unsigned)persistent_blocks(kWPB, 4)),
                               dim3(kBlock), 0, st, W.roff, W.radj, W.nin, W.light, cnt_light,
                               out128, nullptr, nullptr);
        }
        GPM_LAUNCH_CHECK("k_c4_light");
        return GPM_OK;
    }
    hipLaunchKernelGGL(k_degrees, dim3(grid_for(n, 256, 8)), dim3(256), 0, st, g->off, n, W.deg);
    hipLaunchKernelGGL(k_c4_work, dim3(grid_for(n, kWPB, 16)), dim3(kBlock), 0, st, g->off,
                       g->adj, W.deg, n, W.cls);
    GPM_LAUNCH_CHECK("k_c4_work");
    gpm_status rc = split_classes();
    if (rc) return rc;
    const int32_t nparts = (n + kPartZ - 1) / kPartZ;
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
