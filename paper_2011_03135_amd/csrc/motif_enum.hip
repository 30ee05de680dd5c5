// Pattern-oblivious k-motif counting, k = 3, 4, 5 (Section 2 problem 4;
// Section 4 high-level Sandslash: vertex extension of canonical embeddings,
// embedding connectivity codes, classification of each finished embedding
// by its code).  Every connected vertex-induced k-subgraph is enumerated
// exactly once and added to the counter of its isomorphism class.
//
// Canonical embeddings (Appendix B.1: an automorphism check keeps one
// embedding per vertex set).  An embedding is a vertex sequence
// (v0, ..., v_{l-1}).  It may be extended by u iff u > v0 and, with i the
// first position whose vertex is adjacent to u, u is larger than every
// vertex after position i.  Each connected vertex set then has exactly one
// canonical sequence: v0 is its minimum and every later vertex is forced.
// The rule turns into range cuts on sorted rows: the extensions whose first
// neighbour is v_i are the part of N(v_i) above max(v0, v_{i+1}, ...),
// minus the neighbours of v_0..v_{i-1}.
//
// Connectivity codes (Section 4, memoised embedding connectivity;
// Appendix B.6's example): the vertex added at position l contributes l bits,
// bit j set iff it is adjacent to v_j; the embedding's code is the
// concatenation (pair (j, l) at bit l(l-1)/2 + j, 10 bits for k = 5).  The
// prefix for positions below l is kept with the embedding, so only the new
// vertex's bits are computed at each step; a host table maps a full code to
// its motif class.
//
// Kernels.  Positions 0 and 1 are the arcs v0 -> v1 (v1 > v0) of the
// symmetric CSR.  A first pass counts, per arc, the 64-candidate chunks of
// position 2 below it; their exclusive scan numbers the work units (arc,
// chunk), so one arc's work is spread over many waves.  A wave takes a
// unit, binary-searches its arc and searches depth first below the chunk
// with a per-wave stack in LDS.  A level's candidates are the
// concatenation of its (up to k - 1) allowed row ranges; lanes take 64
// candidates at a time, look each one up in the rows of the embedding's
// other vertices (binary search) to get its code bits and drop those whose
// first neighbour is earlier, and the survivors form a lane mask.  At the
// last level the lanes' codes are tallied per distinct code into per-wave
// class counters; otherwise the wave descends into the survivors one by one.
#include <algorithm>
#include <cstdlib>
#include <mutex>
#include <vector>

#include "gpm_internal.h"

namespace gpm {

namespace {

constexpr int kMeMaxK = 5;
constexpr int kMeNT = 256;
constexpr int kMeWaves = kMeNT / kWave;
constexpr int kMeCodes = 1 << (kMeMaxK * (kMeMaxK - 1) / 2);
constexpr int kMeMaxClass = 21;
constexpr int32_t kMncMaxN = 16384;   // graphs up to this size keep a connectivity map per wave

struct MotifEnumPlan {
    uint8_t cls[kMeCodes];   // motif class of each embedding code (0xff: not a code)
};

__device__ __forceinline__ void me_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ bool me_row_has(const int32_t *__restrict__ off,
                                           const int32_t *__restrict__ adj, int32_t u,
                                           int32_t v) {
    int32_t lo = off[u];
    const int32_t end = off[u + 1];
    int32_t hi = end;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (adj[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo < end && adj[lo] == v;
}

__device__ __forceinline__ int32_t me_lower(const int32_t *__restrict__ adj, int32_t lo,
                                            int32_t hi, int32_t x) {
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (adj[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

struct MeWave {
    int32_t m[kMeMaxK];                  // embedding vertex per position
    uint32_t code[kMeMaxK + 1];          // code of positions 0..l-1, kept per level l
    int32_t lo[kMeMaxK][kMeMaxK];        // level l, source i: first allowed index of N(v_i)
    int32_t cum[kMeMaxK][kMeMaxK + 1];   // level l: running lengths of the sources
    int32_t pos[kMeMaxK];                // level l: next candidate of the concatenation
    int32_t lim[kMeMaxK];                // level l: end of the candidates this unit covers
    uint64_t mask[kMeMaxK];              // survivors of the current chunk not yet descended
    int32_t cand[kMeMaxK][kWave];
    uint32_t bits[kMeMaxK][kWave];       // their code bits (bit j: adjacent to v_j)
    unsigned long long cnt[kMeMaxClass];
};

// The row of arc a of a CSR: the last r with off[r] <= a.
__device__ __forceinline__ int32_t me_arc_row(const int32_t *__restrict__ off, int32_t n,
                                              int64_t a) {
    int32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (off[mid] <= a) lo = mid; else hi = mid;
    }
    return lo;
}

// Per arc v0 -> v1 of the symmetric CSR: the number of 64-candidate chunks
// of position 2 below the embedding (v0, v1), 0 unless v1 > v0.
__global__ void k_me_chunks(const int32_t *__restrict__ off, const int32_t *__restrict__ adj,
                            int32_t n, int32_t *__restrict__ chunks) {
    const int64_t narcs = off[n];
    for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < narcs;
         a += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = me_arc_row(off, n, a), v1 = adj[a];
        int32_t c = 0;
        if (v1 > r) {
            const int32_t e0 = off[r + 1], e1 = off[v1 + 1];
            const int32_t t = (e0 - me_lower(adj, off[r], e0, v1 + 1)) +
                              (e1 - me_lower(adj, off[v1], e1, r + 1));
            c = (t + kWave - 1) / kWave;
        }
        chunks[a] = c;
    }
}

template <int K, bool MNC>
__global__ void __launch_bounds__(kMeNT) k_motif_enum(const int32_t *__restrict__ off,
                                                      const int32_t *__restrict__ adj, int32_t n,
                                                      const int64_t *__restrict__ chunk_off,
                                                      unsigned long long *cursor,
                                                      MotifEnumPlan P, int32_t nclass,
                                                      int32_t map_stride,
                                                      unsigned long long *counts) {
    constexpr int kCodes = 1 << (K * (K - 1) / 2);
    __shared__ MeWave sw[kMeWaves];
    __shared__ uint8_t cls[kCodes];
    extern __shared__ uint32_t me_maps[];   // MNC: kMeWaves maps of map_stride words
    const int lane = lane_id(), wib = threadIdx.x / kWave;
    MeWave &S = sw[wib];
    uint32_t *map = me_maps + (size_t)wib * map_stride;
    for (int i = threadIdx.x; i < kCodes; i += kMeNT) cls[i] = P.cls[i];
    if (lane < kMeMaxClass) S.cnt[lane] = 0ull;
    if (MNC)
        for (int i = lane; i < map_stride; i += kWave) map[i] = 0;
    __syncthreads();
    const int64_t nwaves = (int64_t)gridDim.x * kMeWaves;
    const int64_t wave0 = (int64_t)blockIdx.x * kMeWaves + wib;
    const int64_t narcs = off[n];
    const int64_t nchunks = chunk_off[narcs];

    // opens level l of the current embedding: the allowed range of every
    // source row (lane i computes source i), then their running lengths
    auto open_level = [&](int l) {
        if (lane < l) {
            int32_t mx = S.m[0];
            for (int j = lane + 1; j < l; j++) mx = max(mx, S.m[j]);
            const int32_t vi = S.m[lane];
            const int32_t hi = off[vi + 1];
            const int32_t lo = me_lower(adj, off[vi], hi, mx + 1);
            S.lo[l][lane] = lo;
            S.cum[l][lane + 1] = hi - lo;
        }
        me_wave_sync();
        if (lane == 0) {
            int32_t c = 0;
            S.cum[l][0] = 0;
            for (int i = 0; i < l; i++) {
                c += S.cum[l][i + 1];
                S.cum[l][i + 1] = c;
            }
            S.pos[l] = 0;
            S.lim[l] = c;
            S.mask[l] = 0ull;
        }
        me_wave_sync();
    };

    // Connectivity map (MNC): a 4-bit entry per vertex, 8 to a word; bit j
    // of w's entry is set iff w is adjacent to the vertex at position j
    // (positions 0..3 are the ones a later vertex can look back to), kept
    // for the placed positions only.  Neighbouring ids share a word, so the
    // updates are LDS atomics.
    auto mark = [&](int32_t v, uint32_t bit, bool set) {
        const int32_t e = off[v + 1];
        for (int32_t i = off[v] + lane; i < e; i += kWave) {
            const int32_t w = adj[i];
            const uint32_t b = bit << ((w & 7) * 4);
            if (set) atomicOr(map + (w >> 3), b);
            else atomicAnd(map + (w >> 3), ~b);
        }
        me_wave_sync();
    };

    // A work unit is a run of G consecutive chunks (64 candidates of
    // position 2 below one arc, with everything below them).  Units are
    // taken in a fixed interleave for k = 3, whose chunks are single steps,
    // and one chunk at a time from an atomic cursor otherwise (subtrees
    // differ widely).
    constexpr int64_t G = K == 3 ? 32 : 1;
    for (int64_t t = 0;; t++) {
        int64_t unit;
        if (K == 3) {
            unit = t * nwaves + wave0;
        } else {
            unsigned long long got = 0;
            if (lane == 0) got = atomicAdd(cursor, 1ull);
            unit = (int64_t)__shfl(got, 0);
        }
        int64_t c = unit * G;
        if (c >= nchunks) break;   // wave-uniform
        const int64_t c_end = min(c + G, nchunks);
        // the arc of chunk c: the last a with chunk_off[a] <= c
        int64_t a;
        {
            int64_t lo = 0, hi = narcs;
            while (hi - lo > 1) {
                const int64_t mid = (lo + hi) >> 1;
                if (chunk_off[mid] <= c) lo = mid; else hi = mid;
            }
            a = lo;
        }
        int32_t r = me_arc_row(off, n, a);
        for (;;) {
            while (chunk_off[a + 1] <= c) a++;   // arcs without candidates
            if (a >= off[r + 1]) r = me_arc_row(off, n, a);
            const int64_t a_end = min(c_end, chunk_off[a + 1]);
            if (lane == 0) {
                S.m[0] = r;
                S.m[1] = adj[a];
                S.code[2] = 1u;   // v1 ~ v0
            }
            me_wave_sync();
            if (MNC) {
                mark(S.m[0], 1u, true);
                mark(S.m[1], 2u, true);
            }
            open_level(2);
            if (lane == 0) {
                S.pos[2] = (int32_t)(c - chunk_off[a]) * kWave;
                S.lim[2] = min(S.lim[2], (int32_t)(a_end - chunk_off[a]) * kWave);
            }
            me_wave_sync();
            int l = 2;
            while (l >= 2) {
                uint64_t msk = S.mask[l];
                if (msk == 0ull) {
                    const int32_t p = S.pos[l];
                    if (p >= S.lim[l]) {
                        l--;
                        if (MNC && l >= 2) mark(S.m[l], 1u << l, false);
                        continue;
                    }
                    const int32_t q = p + lane;
                    bool valid = q < S.lim[l];
                    int src = 0;
                    for (int i = 1; i < l; i++)
                        if (q >= S.cum[l][i]) src = i;
                    const int32_t u = valid ? adj[S.lo[l][src] + (q - S.cum[l][src])] : 0;
                    uint32_t b = 1u << src;
                    if (MNC) {
                        if (valid) b = (map[u >> 3] >> ((u & 7) * 4)) & ((1u << l) - 1u);
                        // an earlier first neighbour
                        if (b & ((1u << src) - 1u)) valid = false;
                    } else {
                        for (int j = 0; j < l; j++) {
                            if (j == src || !valid) continue;
                            if (me_row_has(off, adj, S.m[j], u)) {
                                if (j < src) valid = false;   // an earlier first neighbour
                                else b |= 1u << j;
                            }
                        }
                    }
                    if (lane == 0) S.pos[l] = p + kWave;
                    uint64_t vm = __ballot(valid);
                    if (l == K - 1) {
                        const uint32_t pre = S.code[l];
                        const int sh = l * (l - 1) / 2;
                        while (vm) {
                            const int fl = __builtin_ctzll(vm);
                            const uint32_t bb = __builtin_amdgcn_readlane(b, fl);
                            const uint64_t same = __ballot(valid && b == bb);
                            vm &= ~same;
                            const int cc = cls[pre | (bb << sh)];
                            if (lane == 0 && cc < kMeMaxClass) S.cnt[cc] += (uint64_t)__popcll(same);
                        }
                        me_wave_sync();
                        continue;
                    }
                    S.cand[l][lane] = u;
                    S.bits[l][lane] = b;
                    if (lane == 0) S.mask[l] = vm;
                    me_wave_sync();
                    msk = vm;
                    if (msk == 0ull) continue;
                }
                // descend into the next survivor of level l
                const int cs = __builtin_ctzll(msk);
                if (lane == 0) {
                    S.mask[l] = msk & (msk - 1ull);
                    S.m[l] = S.cand[l][cs];
                    S.code[l + 1] = S.code[l] | (S.bits[l][cs] << (l * (l - 1) / 2));
                }
                me_wave_sync();
                if (MNC) mark(S.m[l], 1u << l, true);
                l++;
                open_level(l);
            }
            me_wave_sync();
            if (MNC) {
                mark(S.m[0], 1u, false);
                mark(S.m[1], 2u, false);
            }
            c = a_end;
            if (c >= c_end) break;
        }
    }
    __syncthreads();
    if (threadIdx.x < nclass) {
        unsigned long long sum = 0;
        for (int w = 0; w < kMeWaves; w++) sum += sw[w].cnt[threadIdx.x];
        if (sum) atomicAdd(counts + threadIdx.x, sum);
    }
}

// ------------------------------------------------------------- catalogue --
// Motif classes of size k, as canonical codes: the smallest code of the
// class's graphs over all vertex orders.  k = 3 and 4 keep the order of the
// local-counting entry point; k = 5 sorts by edge count, then canonical code.

int pair_bit(int j, int l) { return l * (l - 1) / 2 + j; }   // j < l

uint32_t canon_code(int k, uint32_t code) {
    int perm[kMeMaxK];
    for (int i = 0; i < k; i++) perm[i] = i;
    uint32_t best = ~0u;
    do {
        uint32_t c = 0;
        for (int l = 1; l < k; l++)
            for (int j = 0; j < l; j++) {
                const int a = std::min(perm[j], perm[l]), b = std::max(perm[j], perm[l]);
                if ((code >> pair_bit(a, b)) & 1u) c |= 1u << pair_bit(j, l);
            }
        best = std::min(best, c);
    } while (std::next_permutation(perm, perm + k));
    return best;
}

bool code_connected(int k, uint32_t code) {
    uint32_t seen = 1u, frontier = 1u;
    while (frontier) {
        uint32_t next = 0;
        for (int x = 0; x < k; x++) {
            if (!((frontier >> x) & 1u)) continue;
            for (int y = 0; y < k; y++)
                if (x != y && ((code >> pair_bit(std::min(x, y), std::max(x, y))) & 1u)) next |= 1u << y;
        }
        frontier = next & ~seen;
        seen |= next;
    }
    return seen == (1u << k) - 1u;
}

uint32_t edges_code(int k, std::initializer_list<std::pair<int, int>> e) {
    uint32_t c = 0;
    for (auto &p : e) c |= 1u << pair_bit(std::min(p.first, p.second), std::max(p.first, p.second));
    return canon_code(k, c);
}

// Canonical codes of the classes, in output order.
const std::vector<uint32_t> &motif_catalogue(int k) {
    static const std::vector<uint32_t> c3 = {
        edges_code(3, {{0, 1}, {0, 2}}),                    // wedge
        edges_code(3, {{0, 1}, {0, 2}, {1, 2}}),            // triangle
    };
    static const std::vector<uint32_t> c4 = {
        edges_code(4, {{0, 1}, {0, 2}, {0, 3}}),                            // 3-star
        edges_code(4, {{0, 1}, {1, 2}, {2, 3}}),                            // 4-path
        edges_code(4, {{0, 1}, {1, 2}, {2, 3}, {3, 0}}),                    // 4-cycle
        edges_code(4, {{0, 1}, {0, 2}, {1, 2}, {2, 3}}),                    // tailed triangle
        edges_code(4, {{0, 1}, {0, 2}, {1, 2}, {1, 3}, {2, 3}}),            // diamond
        edges_code(4, {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}}),    // 4-clique
    };
    static const std::vector<uint32_t> c5 = [] {
        std::vector<uint32_t> v;
        for (uint32_t c = 0; c < (1u << 10); c++)
            if (code_connected(5, c) && canon_code(5, c) == c) v.push_back(c);
        std::sort(v.begin(), v.end(), [](uint32_t a, uint32_t b) {
            const int ea = __builtin_popcount(a), eb = __builtin_popcount(b);
            return ea != eb ? ea < eb : a < b;
        });
        return v;
    }();
    return k == 3 ? c3 : k == 4 ? c4 : c5;
}

// cls[code] for every code of a k-vertex embedding.
void make_table(int k, MotifEnumPlan &P) {
    const auto &cat = motif_catalogue(k);
    std::fill(P.cls, P.cls + kMeCodes, (uint8_t)0xff);
    for (uint32_t c = 0; c < (1u << (k * (k - 1) / 2)); c++) {
        if (!code_connected(k, c)) continue;
        const uint32_t cc = canon_code(k, c);
        for (size_t i = 0; i < cat.size(); i++)
            if (cat[i] == cc) P.cls[c] = (uint8_t)i;
    }
}

}  // namespace

int motif_classes(int k) {
    return (k >= 3 && k <= kMeMaxK) ? (int)motif_catalogue(k).size() : 0;
}

gpm_status motif_class_pattern(int k, int idx, gpm_pattern *out) {
    if (k < 3 || k > kMeMaxK) return fail(GPM_UNSUPPORTED, "motif size must be 3, 4 or 5");
    const auto &cat = motif_catalogue(k);
    if (idx < 0 || idx >= (int)cat.size()) return fail(GPM_INVALID_ARGUMENT, "motif index out of range");
    *out = gpm_pattern{};
    out->k = k;
    out->flags = GPM_VERTEX_INDUCED;
    for (int l = 1; l < k; l++)
        for (int j = 0; j < l; j++)
            if ((cat[idx] >> pair_bit(j, l)) & 1u) {
                out->edges[out->n_edges][0] = j;
                out->edges[out->n_edges][1] = l;
                out->n_edges++;
            }
    return GPM_OK;
}

static void me_layout(Carve &cv, int64_t narcs, int32_t **chunks, int64_t **chunk_off,
                      int64_t **tmp, unsigned long long **cursor) {
    *chunks = cv.take<int32_t>((uint64_t)std::max<int64_t>(narcs, 1));
    *chunk_off = cv.take<int64_t>((uint64_t)narcs + 1);
    *tmp = cv.take<int64_t>(scan_tmp_words((uint64_t)narcs));
    *cursor = cv.take<unsigned long long>(1);
}

gpm_status motif_enum_workspace_bytes(const gpm_graph *g, uint64_t *bytes) {
    Carve cv(nullptr, 0);
    int32_t *a;
    int64_t *b, *c;
    unsigned long long *d;
    me_layout(cv, 2 * g->m, &a, &b, &c, &d);
    *bytes = cv.used;
    return GPM_OK;
}

gpm_status motif_enum_count(const gpm_graph *g, int k, void *ws, uint64_t ws_bytes,
                            unsigned long long *out, hipStream_t st) {
    static MotifEnumPlan plans[kMeMaxK + 1];
    static bool made[kMeMaxK + 1] = {};
    static std::mutex mu;
    {
        std::lock_guard<std::mutex> lock(mu);
        if (!made[k]) {
            make_table(k, plans[k]);
            made[k] = true;
        }
    }
    const int64_t narcs = 2 * g->m;
    Carve cv(ws, ws_bytes);
    int32_t *chunks;
    int64_t *chunk_off, *tmp;
    unsigned long long *cursor;
    me_layout(cv, narcs, &chunks, &chunk_off, &tmp, &cursor);
    if (!cv.fits()) return fail(GPM_OUT_OF_MEMORY, "workspace smaller than required");
    const int nclass = motif_classes(k);
    GPM_HIP(fill_u32(reinterpret_cast<uint32_t *>(out), 0, 2 * (uint64_t)nclass, st));
    if (g->m == 0) return GPM_OK;
    Span sp("k_motif_enum", st);
    GPM_HIP(fill_u32(cursor, 0, 2, st));
    const unsigned cblocks = (unsigned)std::min<int64_t>((narcs + 255) / 256, 4096);
    hipLaunchKernelGGL(k_me_chunks, dim3(cblocks), dim3(256), 0, st, g->off, g->adj, g->n, chunks);
    GPM_LAUNCH_CHECK("k_me_chunks");
    GPM_HIP(exclusive_scan_i64(chunks, chunk_off, (uint64_t)narcs, tmp, st));
    // persistent: at most 8 workgroups per CU, fewer for small graphs
    const unsigned blocks = (unsigned)std::max<int64_t>(
        1, std::min<int64_t>((narcs + kMeWaves - 1) / kMeWaves, (int64_t)cu_count() * 8));
    // the connectivity map needs 4 bits per vertex per wave in LDS; k = 3
    // gains nothing from it (its one lookup per candidate is no cheaper than
    // marking the two rows)
    const char *env = getenv("GPM_MNC");
    const bool mnc = k >= 4 && g->n <= kMncMaxN && !(env && env[0] == '0');
    const int32_t stride = mnc ? (g->n + 7) / 8 : 0;   // words
    const size_t dyn = (size_t)kMeWaves * stride * sizeof(uint32_t);
#define ME_LAUNCH(KK, M)                                                                    \
    hipLaunchKernelGGL((k_motif_enum<KK, M>), dim3(blocks), dim3(kMeNT), dyn, st, g->off,  \
                       g->adj, g->n, chunk_off, cursor, plans[k], nclass, stride, out)
    if (k == 3) ME_LAUNCH(3, false);
    else if (k == 4 && mnc) ME_LAUNCH(4, true);
    else if (k == 4) ME_LAUNCH(4, false);
    else if (mnc) ME_LAUNCH(5, true);
    else ME_LAUNCH(5, false);
#undef ME_LAUNCH
    GPM_LAUNCH_CHECK("k_motif_enum");
    return GPM_OK;
}

}  // namespace gpm
