// Counting any connected pattern of up to 6 vertices, vertex- or
// edge-induced (Section 2 problem statement: subgraph listing counts
// edge-induced embeddings, motif counting vertex-induced ones), for the
// patterns the specialised plans do not cover.
//
// Plan (host).  A matching order that keeps every step after the first
// adjacent to an earlier one (greedy: most pattern edges back to the steps
// placed so far, then highest degree), and symmetry-breaking partial orders
// taken from the pattern's automorphism group (Appendix B.1 leaves them to
// the implementation): while the group is not trivial, the first step whose
// vertex v has a non-trivial orbit gets f(v) < f(u) for every other u of
// the orbit, and the group shrinks to v's stabiliser.  Each embedding is
// then matched exactly once.
//
// Kernels.  Steps 0 and 1 are the arcs of the symmetric CSR.  A first pass
// counts, per arc the partial orders accept, the 64-candidate chunks of
// step 2; their exclusive scan numbers the work units (arc, chunk), which
// waves take from an atomic cursor, running the depth-first search below
// the chunk with a per-wave stack in LDS.  At step s >= 2 the candidates
// are a row of the symmetric CSR: that of the already matched backward
// neighbour with the fewest entries, cut by binary search to the range the
// partial orders allow.  Lanes test 64 candidates at a time against the other backward
// neighbours (binary search in their sorted rows), the non-neighbours when
// vertex-induced, and distinctness; the survivors are a lane mask.  At the
// last step the mask's population count is the count; otherwise the wave
// descends into its candidates one by one.
#include <algorithm>
#include <cstdlib>
#include <vector>

#include "gpm_internal.h"

namespace gpm {

namespace {

constexpr int kGenMaxK = 6;
constexpr int kGenMaxE = kGenMaxK * (kGenMaxK - 1) / 2;
constexpr int kGenNT = 256;             // 4 waves per workgroup
constexpr int32_t kGenMncMaxN = 8192;    // graphs up to this size keep a connectivity map per wave

struct GenPlan {
    int32_t k;
    int32_t induced;
    uint32_t back_adj[kGenMaxK];   // earlier steps adjacent to step s in the pattern
    uint32_t back_non[kGenMaxK];   // earlier steps not adjacent to step s
    uint32_t above[kGenMaxK];      // earlier steps t with f(s) > f(t) required
    uint32_t below[kGenMaxK];      // earlier steps t with f(s) < f(t) required
    int32_t vert[kGenMaxK];        // pattern vertex matched at step s (listing rows)
    int32_t dmin[kGenMaxK];        // degree filter: smallest data degree step s accepts
    int32_t ne;                    // pattern edges, as pairs of steps (listing keys)
    int32_t estep[kGenMaxE][2];
};

// Emits one embedding (listing): row f (pattern vertex order, k entries) and
// the checksum term of its key, the ascending vertex tuple (vertex-induced)
// or the ascending edge codes min << 32 | max (edge-induced); m holds the
// data vertex of every step.  May be called from divergent code.
__device__ __forceinline__ void gen_emit(RowEmitter &em, const GenPlan &P,
                                         const int32_t (&m)[kGenMaxK]) {
    int32_t f[kGenMaxK];
    uint64_t key[kGenMaxE];
#pragma unroll
    for (int i = 0; i < kGenMaxE; i++) key[i] = ~0ull;
#pragma unroll
    for (int s = 0; s < kGenMaxK; s++) f[s] = 0;
#pragma unroll
    for (int s = 0; s < kGenMaxK; s++)
        if (s < P.k) {
#pragma unroll
            for (int x = 0; x < kGenMaxK; x++)
                if (x == P.vert[s]) f[x] = m[s];
        }
    int len;
    if (P.induced) {
#pragma unroll
        for (int x = 0; x < kGenMaxK; x++)
            if (x < P.k) key[x] = (uint64_t)(uint32_t)f[x];
        len = P.k;
    } else {
#pragma unroll
        for (int i = 0; i < kGenMaxE; i++)
            if (i < P.ne) {
                uint32_t a = 0, b = 0;
#pragma unroll
                for (int s = 0; s < kGenMaxK; s++) {
                    if (s == P.estep[i][0]) a = (uint32_t)m[s];
                    if (s == P.estep[i][1]) b = (uint32_t)m[s];
                }
                key[i] = a < b ? ((uint64_t)a << 32) | b : ((uint64_t)b << 32) | a;
            }
        len = P.ne;
    }
    // ascending (the padding, all ones, stays at the end)
#pragma unroll
    for (int i = 1; i < kGenMaxE; i++)
#pragma unroll
        for (int j = kGenMaxE - 1; j >= i; j--) {
            const uint64_t x = key[j - 1], y = key[j];
            key[j - 1] = x < y ? x : y;
            key[j] = x < y ? y : x;
        }
    uint64_t h = (uint64_t)len;
#pragma unroll
    for (int i = 0; i < kGenMaxE; i++)
        if (i < len) h = fmix64((h ^ key[i]) + 0x9E3779B97F4A7C15ull);
    em.hsum += h;
    em.count++;
    const uint64_t mask = __ballot(1);
    const int leader = __builtin_ctzll(mask);
    const bool ask = __shfl(em.cached, leader, 64) < em.cap;
    if (!ask) return;
    unsigned long long base = 0;
    if (lane_id() == leader) base = atomicAdd(em.slot_ctr, (unsigned long long)__popcll(mask));
    base = __shfl(base, leader, 64);
    em.cached = base + (uint64_t)__popcll(mask);
    const uint64_t slot = base + (uint64_t)lanes_below(mask);
    if (slot < em.cap) {
        int32_t *o = em.buf + slot * (uint64_t)P.k;
#pragma unroll
        for (int x = 0; x < kGenMaxK; x++)
            if (x < P.k) o[x] = f[x];
    }
}

// Orders a wave's LDS writes before its later reads (lanes of one wave).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ bool row_has(const int32_t *__restrict__ off,
                                        const int32_t *__restrict__ adj, int32_t u, int32_t v) {
    int32_t lo = off[u], hi = off[u + 1];
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (adj[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo < off[u + 1] && adj[lo] == v;
}

// First index in [lo, hi) of the sorted row segment with adj[i] >= x.
__device__ __forceinline__ int32_t lower_idx(const int32_t *__restrict__ adj, int32_t lo,
                                             int32_t hi, int32_t x) {
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (adj[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

struct GenWave {
    int32_t m[kGenMaxK];           // matched vertex per step
    int32_t pos[kGenMaxK], end[kGenMaxK], pivot[kGenMaxK];
    uint64_t mask[kGenMaxK];       // candidates of the current chunk not yet descended into
    int32_t cand[kGenMaxK][kWave];
};

// The row of arc a of a CSR: the last r with off[r] <= a.
__device__ __forceinline__ int32_t gen_arc_row(const int32_t *__restrict__ off, int32_t n,
                                               int64_t a) {
    int32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (off[mid] <= a) lo = mid; else hi = mid;
    }
    return lo;
}

// Candidates of step 2 below the arc (m0, m1): the row of the backward
// neighbour with fewer entries (the first on a tie), cut by binary search to
// the range the partial orders allow.  The search kernel's step opening
// makes the same choice, so the chunk numbering below matches it.
__device__ __forceinline__ int32_t gen_step2_len(const GenPlan &P, const int32_t *__restrict__ off,
                                                 const int32_t *__restrict__ adj, int32_t m0,
                                                 int32_t m1) {
    const bool b0 = P.back_adj[2] & 1u, b1 = (P.back_adj[2] >> 1) & 1u;
    const int32_t l0 = off[m0 + 1] - off[m0], l1 = off[m1 + 1] - off[m1];
    const int32_t mp = (b0 && (!b1 || l0 <= l1)) ? m0 : m1;
    int32_t lo = off[mp], hi = off[mp + 1];
    if (P.above[2] & 1u) lo = lower_idx(adj, lo, hi, m0 + 1);
    if (P.below[2] & 1u) hi = lower_idx(adj, lo, hi, m0);
    if ((P.above[2] >> 1) & 1u) lo = lower_idx(adj, lo, hi, m1 + 1);
    if ((P.below[2] >> 1) & 1u) hi = lower_idx(adj, lo, hi, m1);
    return max(0, hi - lo);
}

// Per arc of the symmetric CSR (steps 0 and 1): 0 if the partial orders
// between the two steps reject it; else, for two-vertex patterns 1 (the arc
// is a match), otherwise the number of 64-candidate chunks of step 2.
__global__ void k_gen_chunks(const int32_t *__restrict__ off, const int32_t *__restrict__ adj,
                             int32_t n, GenPlan P, int32_t *__restrict__ chunks) {
    const int64_t narcs = off[n];
    for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < narcs;
         a += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = gen_arc_row(off, n, a), v1 = adj[a];
        bool ok = true;
        if ((P.above[1] & 1u) && v1 < r) ok = false;
        if ((P.below[1] & 1u) && v1 > r) ok = false;
        // degree filter (Section 4.3): a data vertex below its pattern
        // vertex's degree cannot take it
        if (ok && P.dmin[0] > 1 && off[r + 1] - off[r] < P.dmin[0]) ok = false;
        if (ok && P.dmin[1] > 1 && off[v1 + 1] - off[v1] < P.dmin[1]) ok = false;
        int32_t c = 0;
        if (ok) c = P.k == 2 ? 1 : (gen_step2_len(P, off, adj, r, v1) + kWave - 1) / kWave;
        chunks[a] = c;
    }
}

// Two-vertex patterns: the count is the number of accepted arcs.
__global__ void k_gen_total(const int64_t *__restrict__ total, unsigned long long *out) {
    if (threadIdx.x == 0) out[0] = (unsigned long long)*total;
}

template <bool MNC, bool LIST>
__global__ void __launch_bounds__(kGenNT) k_generic(const int32_t *__restrict__ off,
                                                    const int32_t *__restrict__ adj, int32_t n,
                                                    GenPlan P, const int64_t *__restrict__ chunk_off,
                                                    unsigned long long *cursor, int32_t map_stride,
                                                    unsigned long long *result, RowEmitter em) {
    __shared__ GenWave sw[kGenNT / kWave];
    extern __shared__ uint32_t gen_maps[];   // MNC: a map of map_stride words per wave
    const int lane = lane_id(), wib = threadIdx.x / kWave;
    GenWave &S = sw[wib];
    uint32_t *map = gen_maps + (size_t)wib * map_stride;
    if (MNC)
        for (int i = lane; i < map_stride; i += kWave) map[i] = 0;
    wave_sync();
    // Connectivity map (Section 4, memoised neighbourhood connectivity): a
    // 4-bit entry per vertex, 8 to a word; bit t of w's entry is set iff w
    // is adjacent to the vertex matched at step t, kept for the matched
    // steps up to 3 (what a 5-vertex pattern's last step looks back to).
    auto mark = [&](int32_t v, uint32_t bit, bool set) {
        const int32_t e = off[v + 1];
        for (int32_t i = off[v] + lane; i < e; i += kWave) {
            const int32_t w = adj[i];
            const uint32_t b = bit << ((w & 7) * 4);
            if (set) atomicOr(map + (w >> 3), b);
            else atomicAnd(map + (w >> 3), ~b);
        }
        wave_sync();
    };
    const int32_t last = P.k - 1;
    const int64_t narcs = off[n];
    const int64_t nchunks = chunk_off[narcs];
    uint64_t count = 0;   // wave-uniform
    // candidates of step s: the allowed range of the smallest backward row
    auto open_step = [&](int32_t s) {
        int32_t best = -1, best_len = 0;
        for (int t = 0; t < s; t++) {
            if (!((P.back_adj[s] >> t) & 1u)) continue;
            const int32_t mt = S.m[t];
            const int32_t len = off[mt + 1] - off[mt];
            if (best < 0 || len < best_len) {
                best = t;
                best_len = len;
            }
        }
        const int32_t mp = S.m[best];
        int32_t lo = off[mp], hi = off[mp + 1];
        for (int t = 0; t < s; t++) {
            if ((P.above[s] >> t) & 1u) lo = lower_idx(adj, lo, hi, S.m[t] + 1);
            if ((P.below[s] >> t) & 1u) hi = lower_idx(adj, lo, hi, S.m[t]);
        }
        if (lane == 0) {
            S.pivot[s] = best;
            S.pos[s] = lo;
            S.end[s] = max(lo, hi);
            S.mask[s] = 0ull;
        }
        wave_sync();
    };
    // a work unit is one 64-candidate chunk of step 2 below one arc (steps
    // 0 and 1), with the whole search below it; units come from an atomic
    // cursor, so a hub's arcs and chunks spread over the grid
    for (;;) {
        unsigned long long got = 0;
        if (lane == 0) got = atomicAdd(cursor, 1ull);
        const int64_t c = (int64_t)__shfl(got, 0);
        if (c >= nchunks) break;   // wave-uniform
        int64_t lo = 0, hi = narcs;   // the arc of unit c: last a with chunk_off[a] <= c
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) >> 1;
            if (chunk_off[mid] <= c) lo = mid; else hi = mid;
        }
        const int64_t a = lo;
        if (lane == 0) {
            S.m[0] = gen_arc_row(off, n, a);
            S.m[1] = adj[a];
        }
        wave_sync();
        if (MNC) {
            mark(S.m[0], 1u, true);
            mark(S.m[1], 2u, true);
        }
        open_step(2);
        if (lane == 0) {
            S.pos[2] += (int32_t)(c - chunk_off[a]) * kWave;
            S.end[2] = min(S.end[2], S.pos[2] + kWave);
        }
        wave_sync();
        int32_t s = 2;
        while (s >= 2) {
            uint64_t msk = S.mask[s];
            if (msk == 0ull) {
                const int32_t p = S.pos[s], e = S.end[s];
                if (p >= e) {
                    s--;
                    if (MNC && s >= 2) mark(S.m[s], 1u << s, false);
                    continue;
                }
                const int32_t i = p + lane;
                const int32_t v = i < e ? adj[i] : -1;
                bool ok = i < e;
                if (ok && P.dmin[s] > 1) ok = off[v + 1] - off[v] >= P.dmin[s];
                const int32_t piv = S.pivot[s];
                if (MNC) {
                    for (int t = 0; t < s; t++) ok = ok && v != S.m[t];
                    if (ok) {
                        const uint32_t bits = (map[v >> 3] >> ((v & 7) * 4)) & ((1u << s) - 1u);
                        ok = (bits & P.back_adj[s]) == P.back_adj[s] &&
                             !(P.induced && (bits & P.back_non[s]));
                    }
                } else {
                    for (int t = 0; t < s && ok; t++) {
                        if (t == piv) continue;
                        const int32_t mt = S.m[t];
                        if (v == mt) {
                            ok = false;
                            break;
                        }
                        if ((P.back_adj[s] >> t) & 1u) ok = row_has(off, adj, mt, v);
                        else if (P.induced && ((P.back_non[s] >> t) & 1u)) ok = !row_has(off, adj, mt, v);
                    }
                }
                msk = __ballot(ok);
                wave_sync();
                if (lane == 0) S.pos[s] = p + kWave;
                if (s == last) {
                    if (LIST) {
                        if (ok) {
                            int32_t mm[kGenMaxK];
#pragma unroll
                            for (int t = 0; t < kGenMaxK; t++) mm[t] = t < s ? S.m[t] : v;
                            gen_emit(em, P, mm);
                        }
                    } else {
                        count += (uint64_t)__popcll(msk);
                    }
                    wave_sync();
                    continue;
                }
                S.cand[s][lane] = v;
                if (lane == 0) S.mask[s] = msk;
                wave_sync();
                if (msk == 0ull) continue;
            }
            // descend into the next candidate of step s
            const int cs = __builtin_ctzll(msk);
            if (lane == 0) {
                S.mask[s] = msk & (msk - 1ull);
                S.m[s] = S.cand[s][cs];
            }
            wave_sync();
            if (MNC) mark(S.m[s], 1u << s, true);
            s++;
            open_step(s);
        }
        wave_sync();
        if (MNC) {
            mark(S.m[0], 1u, false);
            mark(S.m[1], 2u, false);
        }
    }
    if (LIST) row_emitter_flush(em, result);
    else if (lane == 0 && count) atomicAdd(result, (unsigned long long)count);
}

// Listing of two-vertex patterns: every arc the partial orders accept.
__global__ void k_gen_list2(const int32_t *__restrict__ off, const int32_t *__restrict__ adj,
                            int32_t n, GenPlan P, unsigned long long *result, RowEmitter em) {
    const int64_t narcs = off[n];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // every lane runs the same number of iterations (the flush is wave-wide)
    for (int64_t a0 = (int64_t)blockIdx.x * blockDim.x; a0 < narcs; a0 += stride) {
        const int64_t a = a0 + threadIdx.x;
        if (a < narcs) {
            const int32_t r = gen_arc_row(off, n, a), v1 = adj[a];
            bool ok = true;
            if ((P.above[1] & 1u) && v1 < r) ok = false;
            if ((P.below[1] & 1u) && v1 > r) ok = false;
            if (ok) {
                int32_t mm[kGenMaxK] = {r, v1};
                gen_emit(em, P, mm);
            }
        }
    }
    row_emitter_flush(em, result);
}

__global__ void k_gen_finish_list(unsigned long long *result, uint64_t cap) {
    if (threadIdx.x == 0) result[1] = result[0] < cap ? result[0] : cap;
}

// ------------------------------------------------------------ planning --

bool connected(int k, const bool (&a)[8][8]) {
    int seen = 1, stack[8], sp = 0;
    stack[sp++] = 0;
    while (sp) {
        const int x = stack[--sp];
        for (int y = 0; y < k; y++)
            if (a[x][y] && !((seen >> y) & 1)) {
                seen |= 1 << y;
                stack[sp++] = y;
            }
    }
    return seen == (1 << k) - 1;
}

gpm_status make_plan(const gpm_pattern *p, GenPlan &P, int32_t *order_out = nullptr,
                     uint32_t *less_out = nullptr) {
    const int k = p->k;
    if (k < 2 || k > kGenMaxK)
        return fail(GPM_UNSUPPORTED, "general patterns: 2 to 6 vertices");
    if (p->n_edges < k - 1 || p->n_edges > k * (k - 1) / 2)
        return fail(GPM_INVALID_ARGUMENT, "edge count impossible for a connected pattern");
    bool a[8][8] = {};
    int deg[8] = {};
    for (int i = 0; i < p->n_edges; i++) {
        const int x = p->edges[i][0], y = p->edges[i][1];
        if (x < 0 || y < 0 || x >= k || y >= k || x == y)
            return fail(GPM_INVALID_ARGUMENT, "pattern edge endpoint out of range or a loop");
        a[x][y] = a[y][x] = true;
    }
    for (int x = 0; x < k; x++)
        for (int y = 0; y < k; y++) deg[x] += a[x][y];
    if (!connected(k, a)) return fail(GPM_UNSUPPORTED, "the pattern is not connected");
    // automorphisms, as maps on pattern vertices
    std::vector<std::vector<int>> group;
    std::vector<int> perm(k);
    for (int i = 0; i < k; i++) perm[i] = i;
    do {
        bool ok = true;
        for (int x = 0; x < k && ok; x++)
            for (int y = 0; y < k; y++)
                if (a[x][y] != a[perm[x]][perm[y]]) {
                    ok = false;
                    break;
                }
        if (ok) group.push_back(perm);
    } while (std::next_permutation(perm.begin(), perm.end()));
    // symmetry-breaking partial orders (Appendix B.1) from the stabiliser
    // chain, vertices taken by degree (highest first, then lowest id): while
    // the group is not trivial, the first vertex v with a non-trivial orbit
    // gets f(v) < f(u) for every other u of its orbit, and the group shrinks
    // to v's stabiliser.  less[x] = the vertices y with f(x) < f(y).
    int byd[8];
    for (int i = 0; i < k; i++) byd[i] = i;
    std::stable_sort(byd, byd + k, [&](int x, int y) { return deg[x] > deg[y]; });
    uint32_t less[8] = {};
    while (group.size() > 1) {
        int v = -1;
        std::vector<int> orbit;
        for (int i = 0; i < k && v < 0; i++) {
            const int x = byd[i];
            std::vector<int> o;
            for (auto &g : group)
                if (std::find(o.begin(), o.end(), g[x]) == o.end()) o.push_back(g[x]);
            if (o.size() > 1) {
                v = x;
                orbit = o;
            }
        }
        for (int u : orbit)
            if (u != v) less[v] |= 1u << u;
        std::vector<std::vector<int>> stab;
        for (auto &g : group)
            if (g[v] == v) stab.push_back(g);
        group.swap(stab);
    }
    // matching order (Appendix B.3, the greedy it takes from DualSim): every
    // step after the first adjacent to an earlier one; at each step the
    // sub-pattern of the placed vertices plus the candidate with (1) more
    // internal partial orders, then (2) more edges; then (ours) the higher
    // degree, then the lower id.  The first two steps are chosen together:
    // an edge carrying a partial order before any other.
    auto po_between = [&](int x, int y) {
        return (int)(((less[x] >> y) & 1u) + ((less[y] >> x) & 1u));
    };
    int order[8], pos[8];
    bool placed[8] = {};
    {
        int bx = -1, by = -1, bpo = -1, bdeg = -1;
        for (int x = 0; x < k; x++)
            for (int y = 0; y < k; y++) {
                if (x == y || !a[x][y]) continue;
                const int po = po_between(x, y), dg = deg[x] + deg[y];
                // x first: the higher degree of the two (then the lower id)
                if (deg[x] < deg[y] || (deg[x] == deg[y] && x > y)) continue;
                if (po > bpo || (po == bpo && dg > bdeg)) {
                    bx = x;
                    by = y;
                    bpo = po;
                    bdeg = dg;
                }
            }
        order[0] = bx;
        order[1] = k > 1 ? by : -1;
        for (int s = 0; s < (k > 1 ? 2 : 1); s++) {
            pos[order[s]] = s;
            placed[order[s]] = true;
        }
    }
    for (int s = 2; s < k; s++) {
        int best = -1, best_po = -1, best_back = -1;
        for (int x = 0; x < k; x++) {
            if (placed[x]) continue;
            int back = 0, po = 0;
            for (int t = 0; t < s; t++) {
                back += a[x][order[t]];
                po += po_between(x, order[t]);
            }
            if (back == 0) continue;
            if (po > best_po || (po == best_po && back > best_back) ||
                (po == best_po && back == best_back && deg[x] > deg[best])) {
                best = x;
                best_po = po;
                best_back = back;
            }
        }
        order[s] = best;
        pos[best] = s;
        placed[best] = true;
    }
    P = GenPlan{};
    P.k = k;
    P.induced = (p->flags & GPM_VERTEX_INDUCED) != 0;
    // the partial orders as step constraints, checked at the later step
    for (int x = 0; x < k; x++)
        for (int y = 0; y < k; y++)
            if ((less[x] >> y) & 1u) {
                if (pos[y] > pos[x]) P.above[pos[y]] |= 1u << pos[x];
                else P.below[pos[x]] |= 1u << pos[y];
            }
    // degree filter (Section 4.3), unless GPM_DF=0 in the environment
    const char *df_env = getenv("GPM_DF");
    const bool df = !(df_env && df_env[0] == '0');
    for (int s = 0; s < k; s++) P.dmin[s] = df ? deg[order[s]] : 0;
    for (int s = 0; s < k; s++)
        for (int t = 0; t < s; t++) {
            if (a[order[s]][order[t]]) P.back_adj[s] |= 1u << t;
            else P.back_non[s] |= 1u << t;
        }
    for (int s = 0; s < k; s++) P.vert[s] = order[s];
    if (order_out)
        for (int s = 0; s < k; s++) order_out[s] = order[s];
    if (less_out)
        for (int x = 0; x < k; x++) less_out[x] = less[x];
    P.ne = p->n_edges;
    for (int i = 0; i < p->n_edges; i++) {
        P.estep[i][0] = pos[p->edges[i][0]];
        P.estep[i][1] = pos[p->edges[i][1]];
    }
    return GPM_OK;
}

}  // namespace

bool generic_pattern_ok(const gpm_pattern *p) {
    GenPlan P;
    return make_plan(p, P) == GPM_OK;
}

gpm_status generic_describe(const gpm_pattern *p, int32_t *order, uint32_t *less) {
    GenPlan P;
    return make_plan(p, P, order, less);
}

static void gen_layout(Carve &cv, int64_t narcs, int32_t **chunks, int64_t **chunk_off,
                       int64_t **tmp, unsigned long long **cursor) {
    *chunks = cv.take<int32_t>((uint64_t)std::max<int64_t>(narcs, 1));
    *chunk_off = cv.take<int64_t>((uint64_t)narcs + 1);
    *tmp = cv.take<int64_t>(scan_tmp_words((uint64_t)narcs));
    *cursor = cv.take<unsigned long long>(2);   // work cursor, listing slot counter
}

uint64_t generic_workspace_bytes(const gpm_graph *g) {
    Carve cv(nullptr, 0);
    int32_t *a;
    int64_t *b, *c;
    unsigned long long *d;
    gen_layout(cv, 2 * g->m, &a, &b, &c, &d);
    return cv.used;
}

// Counting (list == false: out[0] = the count) or listing (out = {total,
// written, checksum}, rows into buf) of a general pattern.
static gpm_status generic_run(const gpm_graph *g, const gpm_pattern *p, bool list, void *ws,
                              uint64_t ws_bytes, int32_t *buf, uint64_t cap,
                              unsigned long long *out, hipStream_t st) {
    GenPlan P;
    gpm_status rc = make_plan(p, P);
    if (rc) return rc;
    const int64_t narcs = 2 * g->m;
    Carve cv(ws, ws_bytes);
    int32_t *chunks;
    int64_t *chunk_off, *tmp;
    unsigned long long *cursor;
    gen_layout(cv, narcs, &chunks, &chunk_off, &tmp, &cursor);
    if (!cv.fits()) return fail(GPM_OUT_OF_MEMORY, "workspace smaller than required");
    GPM_HIP(fill_u32(reinterpret_cast<uint32_t *>(out), 0, list ? 6 : 2, st));
    if (g->m == 0) return GPM_OK;
    Span sp(list ? "k_generic_list" : "k_generic", st);
    GPM_HIP(fill_u32(cursor, 0, 4, st));
    RowEmitter em{cursor + 1, buf, list ? cap : 0, 0, 0, 0};
    const unsigned cblocks = (unsigned)std::min<int64_t>((narcs + 255) / 256, 4096);
    if (list && P.k == 2) {
        hipLaunchKernelGGL(k_gen_list2, dim3(cblocks), dim3(256), 0, st, g->off, g->adj, g->n, P,
                           out, em);
        GPM_LAUNCH_CHECK("k_gen_list2");
        hipLaunchKernelGGL(k_gen_finish_list, dim3(1), dim3(64), 0, st, out, cap);
        GPM_LAUNCH_CHECK("k_gen_finish_list");
        return GPM_OK;
    }
    hipLaunchKernelGGL(k_gen_chunks, dim3(cblocks), dim3(256), 0, st, g->off, g->adj, g->n, P,
                       chunks);
    GPM_LAUNCH_CHECK("k_gen_chunks");
    GPM_HIP(exclusive_scan_i64(chunks, chunk_off, (uint64_t)narcs, tmp, st));
    if (P.k == 2) {
        hipLaunchKernelGGL(k_gen_total, dim3(1), dim3(64), 0, st, chunk_off + narcs, out);
        GPM_LAUNCH_CHECK("k_gen_total");
        return GPM_OK;
    }
    // persistent: at most 8 workgroups per CU, fewer for small graphs
    const unsigned blocks = (unsigned)std::max<int64_t>(
        1, std::min<int64_t>((narcs + kGenNT / kWave - 1) / (kGenNT / kWave),
                             (int64_t)cu_count() * 8));
    // the connectivity map: 4 bits per vertex per wave in LDS, for patterns
    // of at most 5 vertices on graphs of at most 8192 vertices (larger maps
    // cost more occupancy than the searches they save)
    const char *env = getenv("GPM_MNC");
    const bool mnc = P.k <= 5 && g->n <= kGenMncMaxN && !(env && env[0] == '0');
    const int32_t stride = mnc ? (g->n + 7) / 8 : 0;
    const size_t dyn = mnc ? (size_t)(kGenNT / kWave) * stride * sizeof(uint32_t) : 0;
#define GEN_LAUNCH(M, L)                                                                       \
    hipLaunchKernelGGL((k_generic<M, L>), dim3(blocks), dim3(kGenNT), dyn, st, g->off, g->adj,  \
                       g->n, P, chunk_off, cursor, stride, out, em)
    if (mnc && list) GEN_LAUNCH(true, true);
    else if (mnc) GEN_LAUNCH(true, false);
    else if (list) GEN_LAUNCH(false, true);
    else GEN_LAUNCH(false, false);
#undef GEN_LAUNCH
    GPM_LAUNCH_CHECK("k_generic");
    if (list) {
        hipLaunchKernelGGL(k_gen_finish_list, dim3(1), dim3(64), 0, st, out, cap);
        GPM_LAUNCH_CHECK("k_gen_finish_list");
    }
    return GPM_OK;
}

gpm_status generic_count(const gpm_graph *g, const gpm_pattern *p, void *ws, uint64_t ws_bytes,
                         unsigned long long *out, hipStream_t st) {
    return generic_run(g, p, false, ws, ws_bytes, nullptr, 0, out, st);
}

gpm_status generic_list(const gpm_graph *g, const gpm_pattern *p, void *ws, uint64_t ws_bytes,
                        int32_t *buf, uint64_t cap, unsigned long long *result, hipStream_t st) {
    return generic_run(g, p, true, ws, ws_bytes, buf, cap, result, st);
}

}  // namespace gpm
