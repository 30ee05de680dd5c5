// Triangle and k-clique counting/listing on the degree-ordered DAG.
//
// Every k-clique {x_0 < x_1 < ... < x_{k-1}} (in degree order) is found
// exactly once, from x_0, as a path of the DAG: C_1 = N+(x_0), and
// C_{i+1} = C_i ∩ N+(x_i) are the candidates for x_{i+1} (Appendix B.2
// orientation; Appendix B.4 clique pruning; Section 5 local graph).
// Vertices with fewer than k-1 out-neighbours are skipped (degree
// filtering, Section 4.3).
//
// Kernels:
//   k_tc_block      triangles.  The work of root u is the list of pairs
//                   (v, w), v in N+(u), w in N+(v); all pairs of the roots of
//                   one out-degree class form one flattened index space cut
//                   into fixed-size chunks that blocks pop from an atomic
//                   cursor, so a hub's pairs are shared among many blocks.
//                   N+(u) sits in LDS as a hash table next to the pair
//                   prefix of its out-neighbours; each pair is a membership
//                   test of w in N+(u).  Optionally adds 1 to the triangle
//                   count of each of the triangle's three arcs.
//   k_clique_wave   k = 4..9, roots with out-degree <= 64: one wave builds
//                   the local graph on N+(u) as 64-bit adjacency rows in LDS
//                   and counts cliques with AND + popcount.
//   (local_graph.hip) k = 4..9, roots with out-degree 65..1024: workgroup
//                   local graphs in LDS.
//   k_clique_generic  any k in [3, 9] when an out-degree exceeds 1024, and
//                   listing: one wave per root, depth-first with candidate
//                   sets in a per-wave global scratch, wave-cooperative
//                   intersections.
#include "gpm_internal.h"

#include <algorithm>
#include <climits>
#include <cstdlib>

namespace gpm {

gpm_status lg_workspace_bytes(const gpm_graph *g, int32_t k, uint64_t *bytes);
gpm_status lg_cliques(const gpm_graph *g, int32_t k, const int32_t *list_m, const int32_t *cnt_m,
                      const int32_t *list_b, const int32_t *cnt_b, void *ws, uint64_t ws_bytes,
                      unsigned long long *res, unsigned long long *res3,
                      unsigned long long *res4, const RowEmitter *em, hipStream_t st);

namespace {

constexpr int kBlock = 256;
constexpr int kWPB = kBlock / kWave;   // waves per block

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// First index i in [0, n) with a[i] >= x (n if none).
__device__ __forceinline__ int lower_bound_i32(const int32_t *a, int n, int32_t x) {
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Largest j in [0, n) with a[j] <= x, for ascending a with a[0] <= x.
__device__ __forceinline__ int last_le_i32(const int32_t *a, int n, int32_t x) {
    int lo = 0, hi = n;  // invariant: a[lo] <= x
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (a[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ int64_t last_le_i64(const int64_t *a, int64_t n, int64_t x) {
    int64_t lo = 0, hi = n;
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) >> 1;
        if (a[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

// ------------------------------------------------------------ task build --

// Classes of roots by out-degree.
enum RootClass : int { RC_NONE = 0, RC_SMALL = 1, RC_MID = 2, RC_BIG = 3, RC_HUB = 4 };

// Per root: class and pair work W_u = sum over v in N+(u) of d+(v).  Roots
// above big_max are hubs (their arcs become tasks of their own; no work sum).
__global__ void __launch_bounds__(kBlock) k_root_work(const int32_t *__restrict__ dag_off,
                                                      const int32_t *__restrict__ dag_adj,
                                                      int32_t n, int32_t min_out, int32_t small_max,
                                                      int32_t mid_max, int32_t big_max,
                                                      int32_t *work, int32_t *cls) {
    const int lane = lane_id();
    const int64_t wave0 = (int64_t)blockIdx.x * kWPB + threadIdx.x / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * kWPB;
    for (int64_t r = wave0; r < n; r += nwaves) {
        const int32_t s = dag_off[r], d = dag_off[r + 1] - s;
        int c = RC_NONE;
        if (d >= min_out && d <= big_max) c = d <= small_max ? RC_SMALL : (d <= mid_max ? RC_MID : RC_BIG);
        if (d >= min_out && d > big_max) {
            if (lane == 0) {
                cls[r] = RC_HUB;
                work[r] = 0;
            }
            continue;
        }
        int64_t w = 0;
        if (c != RC_NONE)
            for (int32_t i = lane; i < d; i += kWave) {
                int32_t v = dag_adj[s + i];
                w += dag_off[v + 1] - dag_off[v];
            }
        w = wave_sum(w);
        if (lane == 0) {
            cls[r] = (c != RC_NONE && w > 0) ? c : RC_NONE;
            work[r] = (int32_t)w;
        }
    }
}

// flag[r] = (cls[r] == want)
__global__ void k_class_flag(const int32_t *cls, int32_t n, int32_t want, int32_t *flag) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) flag[i] = cls[i] == want ? 1 : 0;
}

// Compacts the flagged roots: list[pos[r]] = r, lwork[pos[r]] = work[r].
__global__ void k_compact_roots(const int32_t *cls, const int32_t *pos, const int32_t *work,
                                int32_t n, int32_t want, int32_t *list, int32_t *lwork) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride)
        if (cls[i] == want) {
            list[pos[i]] = (int32_t)i;
            if (lwork) lwork[pos[i]] = work[i];
        }
}

// Chunk map of a flattened pair space: chunk c starts inside active root a
// iff wpre[a] <= c*tau < wpre[a+1]; first[c] = a.
__global__ void k_chunk_map(const int64_t *wpre, const int32_t *pos_total, int64_t tau,
                            int32_t *first, uint32_t *ctl, unsigned long long *total_pairs) {
    const int32_t nact = *pos_total;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (i == 0) {
        ctl[0] = (uint32_t)nact;
        ctl[1] = (uint32_t)((wpre[nact] + tau - 1) / tau);
        *total_pairs = (unsigned long long)wpre[nact];
    }
    for (; i < nact; i += stride) {
        int64_t c0 = (wpre[i] + tau - 1) / tau, c1 = (wpre[i + 1] + tau - 1) / tau;
        for (int64_t c = c0; c < c1; c++) first[c] = (int32_t)i;
    }
}

// ---------------------------------------------------------- triangles ---

// What k_tc_block does with each triangle (u, v, w), u -> v -> w, u -> w.
enum TcMode : int {
    TC_COUNT = 0,   // count only
    TC_ARCS = 1,    // also +1 on the triangle count of each of its three arcs
    TC_LIST = 2,    // list: emit (u, v, w)
};

// Triangles of the roots of one out-degree class (d+(u) <= DMAX), NT
// threads per block.  A block pops a chunk of tau pairs of the class's
// flattened pair space; for each root u the chunk touches it stages, in LDS,
//   pre[j]   the pair prefix over N+(u) (pairs of v_j start at pre[j]),
//   offj[j]  dag_off[v_j] - pre[j], so pair q of segment j is arc offj[j] + q,
//   a hash table of N+(u) (key v_j, value j; load factor <= 1/4);
// then every wave takes a contiguous run of the chunk's pairs of u.  Lane q
// finds its segment by walking forward from the segment of the previous
// tile's last pair (segments are long on power-law graphs, so a tile
// crosses few boundaries) and tests w in N+(u) with the hash.  In TC_ARCS
// mode the two arcs out of u are counted in LDS and flushed once per root
// and chunk; the arc v -> w takes a global atomic.
template <int DMAX, int NT, int MODE, int U>
__global__ void __launch_bounds__(NT) k_tc_block(const int32_t *__restrict__ dag_off,
                                                 const int32_t *__restrict__ dag_adj,
                                                 const int32_t *__restrict__ act,
                                                 const int64_t *__restrict__ wpre,
                                                 const int32_t *__restrict__ first,
                                                 const uint32_t *__restrict__ ctl,
                                                 uint32_t *cursor, int64_t tau,
                                                 unsigned long long *result, uint32_t *te,
                                                 RowEmitter em) {
    constexpr int NW = NT / kWave;
    constexpr int F = DMAX <= 256 ? 16 : 4;   // slots per out-neighbour
    constexpr int H = F * DMAX;
    constexpr int PER = (DMAX + NT - 1) / NT;
    static_assert(DMAX <= 32767, "local indices are kept as int16");
    __shared__ __align__(16) int32_t keys[H];
    __shared__ int16_t vals[MODE == TC_ARCS ? H : 1];
    __shared__ int32_t pre[DMAX + 1];
    __shared__ int32_t offj[DMAX];
    __shared__ uint32_t cnt[MODE == TC_ARCS ? DMAX : 1];
    __shared__ int32_t verts[MODE == TC_LIST ? DMAX : 1];
    __shared__ int32_t s_sum[NW];
    __shared__ uint32_t s_chunk;
    __shared__ unsigned long long s_acc[NW];
    const int tid = threadIdx.x, lane = lane_id(), wid = tid / kWave;
    const int32_t nact = (int32_t)ctl[0];
    const uint32_t nchunks = ctl[1];
    const int64_t total = wpre[nact];
    if (MODE == TC_ARCS)
        for (int i = tid; i < DMAX; i += NT) cnt[i] = 0;
    uint64_t acc = 0;
    for (;;) {
        if (tid == 0) s_chunk = atomicAdd(cursor, 1u);
        __syncthreads();
        const uint32_t c = s_chunk;
        if (c >= nchunks) break;
        int64_t p = (int64_t)c * tau;
        const int64_t p1 = min(p + tau, total);
        int32_t a = first[c];
        while (p < p1) {
            const int64_t w0 = wpre[a], w1 = wpre[a + 1];
            const int32_t u = act[a];
            const int32_t s = dag_off[u], d = dag_off[u + 1] - s;
            const int32_t hb = lds_hash_bits(d, F);
            for (int i = tid; i < (1 << hb); i += NT) keys[i] = -1;
            stage_root<NT, PER>(dag_off, dag_adj, s, d, keys, MODE == TC_ARCS ? vals : nullptr,
                                hb, pre, offj, s_sum, nullptr,
                                MODE == TC_LIST ? verts : nullptr);
            const int32_t q0 = (int32_t)(p - w0);
            const int32_t q1 = (int32_t)(min(p1, w1) - w0);
            // wave wid takes pairs [qa, qz), whole steps except the last
            const int32_t per_wave =
                ((q1 - q0 + NW - 1) / NW + U * kWave - 1) / (U * kWave) * (U * kWave);
            const int32_t qa = min(q1, q0 + wid * per_wave);
            const int32_t qz = min(q1, qa + per_wave);
            if constexpr (MODE == TC_COUNT) {
                const uint64_t c = walk_count<U>(pre, offj, dag_adj, d, qa, qz, keys, hb);
                if (lane == 0) acc += c;
            } else {
                walk_lookup<U>(pre, offj, dag_adj, d, qa, qz, keys, hb,
                        [&](int32_t jj, int32_t e_vw, int32_t w, int32_t slot) {
                    if (slot >= 0) {
                        acc++;
                        if (MODE == TC_ARCS) {
                            atomicAdd(&cnt[jj], 1u);
                            atomicAdd(&cnt[vals[slot]], 1u);
                            atomicAdd(&te[e_vw], 1u);
                        }
                        if (MODE == TC_LIST) {
                            const int32_t tri[3] = {u, verts[jj], w};
                            emit_vertices<3>(em, tri);
                        }
                    }
                });
            }
            __syncthreads();
            if (MODE == TC_ARCS) {
                for (int32_t i = tid; i < d; i += NT) {
                    const uint32_t x = cnt[i];
                    if (x) {
                        atomicAdd(&te[s + i], x);
                        cnt[i] = 0;
                    }
                }
                __syncthreads();
            }
            p = min(p1, w1);
            a++;
        }
    }
    if (MODE == TC_LIST) {
        row_emitter_flush(em, result);
        return;
    }
    acc = wave_sum(acc);
    if (lane == 0) s_acc[wid] = acc;
    __syncthreads();
    if (tid == 0) {
        unsigned long long t = 0;
        for (int q = 0; q < NW; q++) t += s_acc[q];
        if (t) atomicAdd(result, t);
    }
}

// ------------------------------------------- local-graph k-cliques ---

// Number of D-vertex cliques of the local DAG (rows: 64-bit masks, local
// graph on <= 64 vertices) whose vertices all lie in mask.
template <int D>
__device__ __forceinline__ uint64_t cliques_in64(uint64_t mask, const uint64_t *rows) {
    if constexpr (D == 1) {
        return (uint64_t)__popcll(mask);
    } else if constexpr (D == 2) {
        uint64_t c = 0, m = mask;
        while (m) {
            const int j = __builtin_ctzll(m);
            m &= m - 1;
            c += __popcll(mask & rows[j]);
        }
        return c;
    } else {
        uint64_t c = 0, m = mask;
        while (m) {
            const int j = __builtin_ctzll(m);
            m &= m - 1;
            c += cliques_in64<D - 1>(mask & rows[j], rows);
        }
        return c;
    }
}

// Emits every (K)-clique {u, v_i, ...} through local vertex i (row r): the
// (K-2)-cliques of the local DAG inside r, by nested bit loops.  v holds the
// clique's vertices chosen so far (u, v_i, ...), depth = how many.
template <int K, int DEPTH>
__device__ void list_in64(uint64_t mask, const uint64_t *rows, const int32_t *verts,
                          int32_t (&v)[K], RowEmitter &em) {
    uint64_t m = mask;
    while (m) {
        const int j = __builtin_ctzll(m);
        m &= m - 1;
        v[DEPTH] = verts[j];
        if constexpr (DEPTH + 1 == K) {
            emit_vertices<K>(em, v);
        } else {
            list_in64<K, DEPTH + 1>(mask & rows[j], rows, verts, v, em);
        }
    }
}

// K-cliques of the root through local vertex with row r: (K-2)-cliques of
// the local DAG inside r.
template <int K>
__device__ __forceinline__ uint64_t local_count64(uint64_t r, const uint64_t *rows) {
    return cliques_in64<K - 2>(r, rows);
}

// One 64-thread block (one wave) per root at a time: stages N+(u), sets the
// local rows through the pair walk and the membership hash, then counts.
template <int K, bool LIST>
__global__ void __launch_bounds__(kWave) k_clique_wave(const int32_t *__restrict__ dag_off,
                                                       const int32_t *__restrict__ dag_adj,
                                                       const int32_t *__restrict__ roots,
                                                       const int32_t *__restrict__ nroots_p,
                                                       unsigned long long *result,
                                                       unsigned long long *res3,
                                                       unsigned long long *res4, RowEmitter em) {
    __shared__ uint64_t rows[kWave];
    __shared__ __align__(16) int32_t keys[8 * kWave];
    __shared__ int16_t vals[8 * kWave];
    __shared__ int32_t pre[kWave + 1], offj[kWave];
    __shared__ int32_t verts[LIST ? kWave : 1];
    const int lane = lane_id();
    const int32_t nroots = *nroots_p;
    uint64_t acc = 0, acc3 = 0, acc4 = 0;
    for (int64_t r = blockIdx.x; r < nroots; r += gridDim.x) {
        const int32_t u = roots[r];
        const int32_t s = dag_off[u], d = dag_off[u + 1] - s;
        const int32_t hb = lds_hash_bits(d, 8);
        for (int i = lane; i < (1 << hb); i += kWave) keys[i] = -1;
        rows[lane] = 0;
        stage_root<kWave, 1>(dag_off, dag_adj, s, d, keys, vals, hb, pre, offj, nullptr, nullptr,
                             LIST ? verts : nullptr);
        walk_lookup<2>(pre, offj, dag_adj, d, 0, pre[d], keys, hb,
                [&](int32_t j, int32_t, int32_t w, int32_t slot) {
            if (slot >= 0) atomicOr((unsigned long long *)&rows[j], 1ull << vals[slot]);
        });
        __syncthreads();
        if (lane < d) {
            if constexpr (LIST) {
                int32_t v[K];
                v[0] = u;
                v[1] = verts[lane];
                list_in64<K, 2>(rows[lane], rows, verts, v, em);
            } else {
                acc += local_count64<K>(rows[lane], rows);
                if (res3) acc3 += __popcll(rows[lane]);                 // triangles at u
                if (K == 5 && res4) acc4 += local_count64<4>(rows[lane], rows);
            }
        }
        __syncthreads();
    }
    if (LIST) {
        row_emitter_flush(em, result);
        return;
    }
    acc = wave_sum(acc);
    if (lane == 0 && acc) atomicAdd(result, (unsigned long long)acc);
    if (res3) {
        acc3 = wave_sum(acc3);
        if (lane == 0 && acc3) atomicAdd(res3, (unsigned long long)acc3);
    }
    if (K == 5 && res4) {
        acc4 = wave_sum(acc4);
        if (lane == 0 && acc4) atomicAdd(res4, (unsigned long long)acc4);
    }
}

constexpr int kMidMaxD = 256;

// ------------------------------------------------- generic DFS (k <= 9) ---

constexpr int kGenMaxK = 9;

struct ListOut {
    int32_t *buf;
    uint64_t cap;
};

// Wave-cooperative |A ∩ B| or A ∩ B (ascending, into out) for ascending
// global arrays; lanes walk the shorter list and binary-search the longer.
template <bool WRITE>
__device__ int32_t wave_intersect(const int32_t *a, int32_t na, const int32_t *b, int32_t nb,
                                  int32_t *out) {
    const int lane = lane_id();
    if (na > nb) {
        const int32_t *t = a; a = b; b = t;
        int32_t tn = na; na = nb; nb = tn;
    }
    int32_t cnt = 0;
    for (int32_t i0 = 0; i0 < na; i0 += kWave) {
        const int32_t i = i0 + lane;
        bool hit = false;
        int32_t x = 0;
        if (i < na) {
            x = a[i];
            int32_t p = lower_bound_i32(b, nb, x);
            hit = p < nb && b[p] == x;
        }
        const uint64_t mask = __ballot(hit);
        if (WRITE && hit) out[cnt + lanes_below(mask)] = x;
        cnt += __popcll(mask);
    }
    return cnt;
}

__device__ __forceinline__ void sort_small(uint64_t *k, int len) {
    for (int i = 1; i < len; i++) {
        uint64_t x = k[i];
        int j = i - 1;
        while (j >= 0 && k[j] > x) { k[j + 1] = k[j]; j--; }
        k[j + 1] = x;
    }
}

template <bool LIST>
__global__ void __launch_bounds__(kBlock) k_clique_generic(const int32_t *__restrict__ dag_off,
                                                           const int32_t *__restrict__ dag_adj,
                                                           int32_t n, int32_t k, int32_t maxout,
                                                           int32_t *scratch,
                                                           unsigned long long *result,
                                                           ListOut lo) {
    const int lane = lane_id();
    const int64_t wave_gid = (int64_t)blockIdx.x * kWPB + threadIdx.x / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * kWPB;
    int32_t *mine = scratch + wave_gid * (int64_t)(kGenMaxK - 2) * maxout;
    uint64_t acc = 0, hsum = 0;
    const int last = k - 2;   // level whose intersection is counted/listed
    for (int64_t ur = wave_gid; ur < n; ur += nwaves) {
        const int32_t u = (int32_t)ur;
        const int32_t s = dag_off[u], d = dag_off[u + 1] - s;
        if (d < k - 1) continue;
        const int32_t *cand[kGenMaxK];
        int32_t csz[kGenMaxK], it[kGenMaxK], pv[kGenMaxK];
        cand[1] = dag_adj + s;
        csz[1] = d;
        it[1] = 0;
        pv[0] = u;
        int l = 1;
        while (l >= 1) {
            if (it[l] >= csz[l]) {
                l--;
                if (l >= 1) it[l]++;
                continue;
            }
            const int32_t v = cand[l][it[l]];
            pv[l] = v;
            const int32_t vs = dag_off[v], vd = dag_off[v + 1] - vs;
            if (l == last) {
                if (!LIST) {
                    const int32_t c = wave_intersect<false>(cand[l], csz[l], dag_adj + vs, vd, nullptr);
                    if (lane == 0) acc += (uint64_t)c;   // c is wave-uniform
                } else {
                    // enumerate C_l ∩ N+(v): each element closes a k-clique
                    const int32_t *a = cand[l], *b = dag_adj + vs;
                    int32_t na = csz[l], nb = vd;
                    for (int32_t i0 = 0; i0 < na; i0 += kWave) {
                        const int32_t i = i0 + lane;
                        bool hit = false;
                        int32_t x = 0;
                        if (i < na) {
                            x = a[i];
                            int32_t p = lower_bound_i32(b, nb, x);
                            hit = p < nb && b[p] == x;
                        }
                        const uint64_t mask = __ballot(hit);
                        if (!mask) continue;
                        unsigned long long basei = 0;
                        if (lane == 0) basei = atomicAdd(&result[0], (unsigned long long)__popcll(mask));
                        basei = __shfl(basei, 0, 64);
                        if (hit) {
                            uint64_t key[kGenMaxK];
                            for (int t = 0; t <= last; t++) key[t] = (uint64_t)(uint32_t)pv[t];
                            key[last + 1] = (uint64_t)(uint32_t)x;
                            const uint64_t slot = basei + lanes_below(mask);
                            if (slot < lo.cap) {
                                int32_t *o = lo.buf + slot * (uint64_t)k;
                                for (int t = 0; t <= last; t++) o[t] = pv[t];
                                o[last + 1] = x;
                            }
                            sort_small(key, k);
                            uint64_t h = (uint64_t)k;
                            for (int t = 0; t < k; t++) h = fmix64((h ^ key[t]) + 0x9E3779B97F4A7C15ull);
                            hsum += h;
                        }
                    }
                }
                it[l]++;
            } else {
                int32_t *out = mine + (int64_t)(l - 1) * maxout;
                const int32_t c = wave_intersect<true>(cand[l], csz[l], dag_adj + vs, vd, out);
                wave_sync();
                if (c >= k - 1 - l) {
                    l++;
                    cand[l] = out;
                    csz[l] = c;
                    it[l] = 0;
                } else {
                    it[l]++;
                }
            }
        }
    }
    if (!LIST) {
        acc = wave_sum(acc);
        if (lane == 0 && acc) atomicAdd(&result[0], (unsigned long long)acc);
    } else {
        hsum = wave_sum(hsum);
        if (lane == 0) atomicAdd(&result[2], (unsigned long long)hsum);
    }
}

// written = min(slots handed out, cap)
__global__ void k_finish_rows(unsigned long long *result, const unsigned long long *slot_ctr,
                              uint64_t cap) {
    if (threadIdx.x == 0 && blockIdx.x == 0) result[1] = *slot_ctr < cap ? *slot_ctr : cap;
}

__global__ void k_finish_listing(unsigned long long *result, uint64_t cap) {
    if (threadIdx.x == 0 && blockIdx.x == 0) result[1] = result[0] < cap ? result[0] : cap;
}

// ----------------------------------------------- hub roots (d+ > 1024) ---
//
// Roots whose out-degree exceeds the largest class (their N+(u) does not fit
// the LDS staging of the triangle and local-graph kernels) are split at edge
// granularity (Section 4.1's task model): every arc u -> v of such a root is
// a task of its own, taken by one wave from a flattened index space over the
// hub roots' arcs.  The wave intersects N+(u) and N+(v) (lanes walk the
// shorter list and binary-search the longer) into its scratch and searches
// depth first below the result as k_clique_generic does.

enum HubMode : int {
    HUB_COUNT = 0,   // count K-cliques (and triangles / 4-cliques into res3 / res4)
    HUB_ARCS = 1,    // K = 3: count triangles and add 1 per triangle to each of its arcs
    HUB_LIST = 2,    // list K-cliques through the row emitter
};

// Per hub root r (list hubs[0..nh)), its out-degree: the arc counts whose
// scan numbers the tasks.
__global__ void k_hub_arcs(const int32_t *dag_off, const int32_t *hubs, const int32_t *nh_p,
                           int32_t *cnt) {
    const int32_t nh = *nh_p;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nh;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t u = hubs[i];
        cnt[i] = dag_off[u + 1] - dag_off[u];
    }
}

template <int K, int MODE>
__global__ void __launch_bounds__(kBlock) k_clique_hub(const int32_t *__restrict__ dag_off,
                                                       const int32_t *__restrict__ dag_adj,
                                                       const int32_t *__restrict__ hubs,
                                                       const int64_t *__restrict__ hpre,
                                                       const int32_t *__restrict__ nh_p,
                                                       int32_t maxout, int32_t *scratch,
                                                       unsigned long long *res,
                                                       unsigned long long *res3,
                                                       unsigned long long *res4, uint32_t *te,
                                                       RowEmitter em) {
    static_assert(K >= 3 && K <= kGenMaxK, "clique size");
    static_assert(MODE != HUB_ARCS || K == 3, "arc counts are triangle counts");
    const int lane = lane_id();
    const int64_t wave_gid = (int64_t)blockIdx.x * kWPB + threadIdx.x / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * kWPB;
    int32_t *mine = scratch + wave_gid * (int64_t)(kGenMaxK - 2) * maxout;
    const int32_t nh = *nh_p;
    const int64_t total = hpre[nh];
    // fused counts need every 4-clique below an arc, so only K's own
    // pruning applies when no 4-cliques are asked for
    const int32_t need2 = (res4 && K > 4) ? 2 : K - 2;
    uint64_t acc = 0, acc3 = 0, acc4 = 0;
    for (int64_t t = wave_gid; t < total; t += nwaves) {
        const int32_t r = (int32_t)last_le_i64(hpre, (int64_t)nh + 1, t);
        const int32_t u = hubs[r];
        const int32_t s = dag_off[u], d = dag_off[u + 1] - s;
        const int32_t e = s + (int32_t)(t - hpre[r]);
        const int32_t v = dag_adj[e];
        const int32_t vs = dag_off[v], vd = dag_off[v + 1] - vs;
        if constexpr (MODE == HUB_ARCS || (K == 3 && MODE == HUB_LIST)) {
            // every common out-neighbour w closes the triangle (u, v, w)
            const bool u_short = d <= vd;
            const int32_t *a = u_short ? dag_adj + s : dag_adj + vs;
            const int32_t *b = u_short ? dag_adj + vs : dag_adj + s;
            const int32_t na = u_short ? d : vd, nb = u_short ? vd : d;
            uint32_t c = 0;
            for (int32_t i0 = 0; i0 < na; i0 += kWave) {
                const int32_t i = i0 + lane;
                bool hit = false;
                int32_t x = 0, p = 0;
                if (i < na) {
                    x = a[i];
                    p = lower_bound_i32(b, nb, x);
                    hit = p < nb && b[p] == x;
                }
                if (hit) {
                    if constexpr (MODE == HUB_ARCS) {
                        // arcs u -> w and v -> w
                        atomicAdd(&te[(u_short ? s + i : s + p)], 1u);
                        atomicAdd(&te[(u_short ? vs + p : vs + i)], 1u);
                    } else {
                        const int32_t tri[3] = {u, v, x};
                        emit_vertices<3>(em, tri);
                    }
                }
                c += (uint32_t)__popcll(__ballot(hit));
            }
            if (lane == 0) {
                acc += c;
                if (MODE == HUB_ARCS && c) atomicAdd(&te[e], c);   // arc u -> v
            }
            continue;
        } else {
            if constexpr (K == 3) {
                const int32_t c = wave_intersect<false>(dag_adj + s, d, dag_adj + vs, vd, nullptr);
                if (lane == 0) acc += (uint64_t)c;
                continue;
            } else {
                // level 1: C = N+(u) ∩ N+(v), the triangles on the arc
                const int32_t c2 = wave_intersect<true>(dag_adj + s, d, dag_adj + vs, vd, mine);
                wave_sync();
                if (res3 && lane == 0) acc3 += (uint64_t)c2;
                if (c2 < need2) continue;
                const int32_t *cand[kGenMaxK];
                int32_t csz[kGenMaxK], it[kGenMaxK], pv[kGenMaxK];
                pv[0] = u;
                pv[1] = v;
                cand[2] = mine;
                csz[2] = c2;
                it[2] = 0;
                constexpr int last = K - 2;   // level whose intersection is counted or listed
                int l = 2;
                while (l >= 2) {
                    if (it[l] >= csz[l]) {
                        l--;
                        if (l >= 2) it[l]++;
                        continue;
                    }
                    const int32_t w = cand[l][it[l]];
                    pv[l] = w;
                    const int32_t ws = dag_off[w], wd = dag_off[w + 1] - ws;
                    if (l == last) {
                        if constexpr (MODE == HUB_COUNT) {
                            const int32_t c = wave_intersect<false>(cand[l], csz[l], dag_adj + ws,
                                                                    wd, nullptr);
                            if (lane == 0) acc += (uint64_t)c;
                        } else {
                            const int32_t *a = cand[l], *b = dag_adj + ws;
                            const int32_t na = csz[l], nb = wd;
                            for (int32_t i0 = 0; i0 < na; i0 += kWave) {
                                const int32_t i = i0 + lane;
                                if (i < na) {
                                    const int32_t x = a[i];
                                    const int32_t p = lower_bound_i32(b, nb, x);
                                    if (p < nb && b[p] == x) {
                                        int32_t q[K];
#pragma unroll
                                        for (int z = 0; z < K - 1; z++) q[z] = pv[z];
                                        q[K - 1] = x;
                                        emit_vertices<K>(em, q);
                                    }
                                }
                            }
                        }
                        it[l]++;
                    } else {
                        int32_t *out = mine + (int64_t)(l - 1) * maxout;
                        const int32_t c = wave_intersect<true>(cand[l], csz[l], dag_adj + ws, wd,
                                                               out);
                        wave_sync();
                        if (res4 && l == 2 && lane == 0) acc4 += (uint64_t)c;
                        if (c >= K - 1 - l) {
                            l++;
                            cand[l] = out;
                            csz[l] = c;
                            it[l] = 0;
                        } else {
                            it[l]++;
                        }
                    }
                }
            }
        }
    }
    if constexpr (MODE == HUB_LIST) {
        row_emitter_flush(em, res);
        return;
    }
    acc = wave_sum(acc);
    if (lane == 0 && acc) atomicAdd(res, (unsigned long long)acc);
    if (res3) {
        acc3 = wave_sum(acc3);
        if (lane == 0 && acc3) atomicAdd(res3, (unsigned long long)acc3);
    }
    if (res4) {
        acc4 = wave_sum(acc4);
        if (lane == 0 && acc4) atomicAdd(res4, (unsigned long long)acc4);
    }
}

// ------------------------------------------------------------ host side --

// Triangle classes by out-degree: (1, 64] one wave per block, (64, 256] and
// (256, 1024] larger blocks sharing one staged root.  Chunk sizes in pairs
// (per graph, gpm_graph::tc_tau): every chunk costs one atomic on the
// class's cursor, and a few hundred thousand atomics on one address cost
// milliseconds, so chunks stay large; too large, and the last chunks leave
// most of the grid idle.
constexpr int32_t kTcSmall = 64, kTcMid = 256, kTcMax = 1024;

struct CliqueWs {
    unsigned long long *result;   // [8]: count, -, pairs of each triangle class
    uint32_t *ctl;                // [32]: cursors, per-class {nact, nchunks}, class counts
    int32_t *work, *cls, *flag, *pos;
    int32_t *list_s, *list_m, *list_b, *list_h;
    int32_t *lwork;               // compacted work of one class (reused)
    int64_t *wpre_s, *wpre_m, *wpre_b, *wpre_h;
    int32_t *first_s, *first_m, *first_b;
    int64_t *scan_tmp;
    void *lg;                     // local-graph workspace (k = 4, 5)
    uint64_t lg_bytes;
    int32_t *gen_scratch;
    int gen_waves;
    uint64_t bytes;
};

int64_t chunk_bound(const gpm_graph *g) {
    // total pair work = sum_v d-(v) d+(v) <= m * max_out; chunks = ceil(total / tau)
    int64_t w = g->m * (int64_t)std::max(g->max_out_degree, 1);
    const int64_t tau = std::min({g->tc_tau[0], g->tc_tau[1], g->tc_tau[2]});
    return w / std::max<int64_t>(tau, 1) + 2;
}

// The generic DFS (a wave per root) serves listings of k >= 6; every other
// count and listing runs on the triangle and local-graph kernels, with roots
// of out-degree above 1024 split per arc (k_clique_hub).  GPM_LG=0 in the
// environment sends every root of k >= 4 to the per-arc depth-first search
// instead: the search without local graphs, equally load-balanced, for
// comparison.
bool lg_disabled(int32_t k) {
    const char *env = getenv("GPM_LG");
    return k >= 4 && env && env[0] == '0';
}

bool uses_generic(const gpm_graph *g, int32_t k, bool list) {
    (void)g;
    return list && k > 5;
}

// Roots above the largest class go to k_clique_hub.
bool has_hubs(const gpm_graph *g) { return g->max_out_degree > kTcMax; }

bool uses_hub_kernel(const gpm_graph *g, int32_t k) { return has_hubs(g) || lg_disabled(k); }

CliqueWs clique_layout(const gpm_graph *g, int32_t k, bool list, void *base) {
    CliqueWs W{};
    Carve c(base, ~0ull);
    const uint64_t n1 = (uint64_t)g->n + 1;
    W.result = c.take<unsigned long long>(8);
    W.ctl = c.take<uint32_t>(32);
    W.work = c.take<int32_t>(n1);
    W.cls = c.take<int32_t>(n1);
    W.flag = c.take<int32_t>(n1);
    W.pos = c.take<int32_t>(n1);
    W.list_s = c.take<int32_t>(n1);
    W.list_m = c.take<int32_t>(n1);
    W.list_b = c.take<int32_t>(n1);
    W.list_h = c.take<int32_t>(n1);
    W.lwork = c.take<int32_t>(n1);
    W.wpre_s = c.take<int64_t>(n1);
    W.wpre_m = c.take<int64_t>(n1);
    W.wpre_b = c.take<int64_t>(n1);
    W.wpre_h = c.take<int64_t>(n1);
    W.scan_tmp = c.take<int64_t>(scan_tmp_words(n1));
    bool generic = uses_generic(g, k, list);
    if (!generic && k == 3) {
        W.first_s = c.take<int32_t>((uint64_t)chunk_bound(g));
        W.first_m = c.take<int32_t>((uint64_t)chunk_bound(g));
        W.first_b = c.take<int32_t>((uint64_t)chunk_bound(g));
    }
    if (!generic && k >= 4 && !lg_disabled(k)) {
        lg_workspace_bytes(g, k, &W.lg_bytes);
        W.lg = c.take<char>(W.lg_bytes);
    }
    if (generic || uses_hub_kernel(g, k)) {
        W.gen_waves = persistent_blocks(kWPB, 8) * kWPB;
        W.gen_scratch = c.take<int32_t>((uint64_t)W.gen_waves * (kGenMaxK - 2) *
                                        (uint64_t)std::max(1, g->max_out_degree));
    }
    W.bytes = c.used;
    return W;
}

unsigned grid_for(int64_t items, int per_block, int cap_per_cu) {
    int64_t b = (items + per_block - 1) / per_block;
    int64_t cap = (int64_t)cu_count() * cap_per_cu;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

// Builds the compacted root list of one class; returns its count in *count_dev
// (device int32 = pos[n]) and, when wpre is given, the int64 work prefix.
hipError_t build_class(const gpm_graph *g, CliqueWs &W, int32_t want, int32_t *list,
                       int64_t *wpre, hipStream_t st) {
    const int32_t n = g->n;
    if (wpre) {
        hipError_t z = fill_u32(W.lwork, 0, (uint64_t)n + 1, st);
        if (z != hipSuccess) return z;
    }
    hipLaunchKernelGGL(k_class_flag, dim3(grid_for(n, 256, 8)), dim3(256), 0, st, W.cls, n, want,
                       W.flag);
    hipError_t e = exclusive_scan_i32(W.flag, W.pos, (uint64_t)n, W.scan_tmp, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_compact_roots, dim3(grid_for(n, 256, 8)), dim3(256), 0, st, W.cls, W.pos,
                       W.work, n, want, list, wpre ? W.lwork : (int32_t *)nullptr);
    e = hipGetLastError();
    if (e != hipSuccess || !wpre) return e;
    // work prefix over the class's roots; the count is pos[n] (device)
    return exclusive_scan_i64(W.lwork, wpre, (uint64_t)n, W.scan_tmp, st);
}

// Cliques (or, K = 3 with HUB_ARCS, per-arc triangle counts) rooted at the
// hub roots, the roots above the largest class; W.cls must hold the classes
// from k_root_work.  Nothing is launched on graphs without hubs.
template <int K, int MODE>
gpm_status hub_launch(const gpm_graph *g, CliqueWs &W, unsigned long long *res,
                      unsigned long long *res3, unsigned long long *res4, uint32_t *te,
                      const RowEmitter &em, hipStream_t st, bool all_roots = false) {
    if (!has_hubs(g) && !all_roots) return GPM_OK;
    const int32_t n = g->n;
    int32_t *cnt_h = (int32_t *)(W.ctl + 15);
    GPM_HIP(build_class(g, W, RC_HUB, W.list_h, nullptr, st));
    GPM_HIP(hipMemcpyAsync(cnt_h, W.pos + n, 4, hipMemcpyDeviceToDevice, st));
    GPM_HIP(fill_u32(W.lwork, 0, (uint64_t)n + 1, st));
    hipLaunchKernelGGL(k_hub_arcs, dim3(grid_for(n, 256, 8)), dim3(256), 0, st, g->dag_off,
                       W.list_h, cnt_h, W.lwork);
    GPM_LAUNCH_CHECK("k_hub_arcs");
    GPM_HIP(exclusive_scan_i64(W.lwork, W.wpre_h, (uint64_t)n, W.scan_tmp, st));
    {
        static const char *const kNames[] = {"k_clique_hub<3>", "k_clique_hub<4>",
                                             "k_clique_hub<5>", "k_clique_hub<6>",
                                             "k_clique_hub<7>", "k_clique_hub<8>",
                                             "k_clique_hub<9>"};
        Span sp(kNames[K - 3], st);
        hipLaunchKernelGGL((k_clique_hub<K, MODE>), dim3((unsigned)(W.gen_waves / kWPB)),
                           dim3(kBlock), 0, st, g->dag_off, g->dag_adj, W.list_h,
                           (const int64_t *)W.wpre_h, (const int32_t *)cnt_h,
                           std::max(1, g->max_out_degree), W.gen_scratch, res, res3, res4, te,
                           em);
    }
    GPM_LAUNCH_CHECK("k_clique_hub");
    return GPM_OK;
}

template <int K>
gpm_status launch_local(const gpm_graph *g, CliqueWs &W, const int32_t *cnt_s,
                        const int32_t *cnt_m, const int32_t *cnt_b, unsigned long long *res,
                        unsigned long long *res3, unsigned long long *res4, hipStream_t st,
                        const RowEmitter *em = nullptr) {
    gpm_status rc = lg_cliques(g, K, W.list_m, cnt_m, W.list_b, cnt_b, W.lg, W.lg_bytes, res,
                               res3, res4, em, st);
    if (rc) return rc;
    {
        static const char *const kNames[] = {"k_clique_wave<4>", "k_clique_wave<5>",
                                             "k_clique_wave<6>", "k_clique_wave<7>",
                                             "k_clique_wave<8>", "k_clique_wave<9>"};
        Span sp(kNames[K - 4], st);
        if (em)
            hipLaunchKernelGGL((k_clique_wave<K, true>), dim3((unsigned)(cu_count() * g->cw_bpc)),
                               dim3(kWave), 0, st, g->dag_off, g->dag_adj, W.list_s, cnt_s, res,
                               res3, res4, *em);
        else
            hipLaunchKernelGGL((k_clique_wave<K, false>), dim3((unsigned)(cu_count() * g->cw_bpc)),
                               dim3(kWave), 0, st, g->dag_off, g->dag_adj, W.list_s, cnt_s, res,
                               res3, res4, RowEmitter{});
    }
    GPM_LAUNCH_CHECK("k_clique_wave");
    if constexpr (K <= 5) {
        if (em) return hub_launch<K, HUB_LIST>(g, W, res, nullptr, nullptr, nullptr, *em, st);
    }
    return hub_launch<K, HUB_COUNT>(g, W, res, res3, res4, nullptr, RowEmitter{}, st);
}

}  // namespace

gpm_status clique_workspace_bytes(const gpm_graph *g, int32_t k, bool list, uint64_t *bytes) {
    if (k < 3 || k > kGenMaxK) return fail(GPM_UNSUPPORTED, "clique size must be in [3, 9]");
    *bytes = clique_layout(g, k, list, nullptr).bytes;
    return GPM_OK;
}

template <int DMAX, int NT, int MODE>
static gpm_status tc_class(const gpm_graph *g, CliqueWs &W, int32_t want, int32_t *list,
                           int64_t *wpre, int32_t *first, int cls_idx, int64_t tau,
                           int blocks_per_cu, const char *name, unsigned long long *res,
                           uint32_t *te, const RowEmitter &em, hipStream_t st) {
    const int32_t n = g->n;
    uint32_t *info = W.ctl + 4 + 2 * cls_idx;   // {nact, nchunks}
    GPM_HIP(build_class(g, W, want, list, wpre, st));
    hipLaunchKernelGGL(k_chunk_map, dim3(grid_for(n, 256, 8)), dim3(256), 0, st, wpre, W.pos + n,
                       tau, first, info, W.result + 2 + cls_idx);
    GPM_LAUNCH_CHECK("k_chunk_map");
    {
        Span sp(name, st);
        hipLaunchKernelGGL((k_tc_block<DMAX, NT, MODE, MODE == TC_COUNT ? 4 : 2>),
                           dim3((unsigned)(cu_count() * blocks_per_cu)), dim3(NT), 0, st,
                           g->dag_off, g->dag_adj, list, wpre, first, info, W.ctl + cls_idx,
                           tau, res, te, em);
        span_units(W.result + 2 + cls_idx, st);
    }
    GPM_LAUNCH_CHECK(name);
    return GPM_OK;
}

// Triangle count into *res (zero on entry); with MODE == TC_ARCS also adds 1
// to the triangle count of each of the three arcs of every triangle (te, m
// words, zero on entry).  Uses the triangle workspace
// (clique_workspace_bytes(g, 3, false)).
template <int MODE>
static gpm_status tc_launch(const gpm_graph *g, CliqueWs &W, unsigned long long *res,
                            uint32_t *te, hipStream_t st, const RowEmitter &em = RowEmitter{}) {
    const int32_t n = g->n;
    GPM_HIP(fill_u32(W.ctl, 0, 32, st));
    hipLaunchKernelGGL(k_root_work, dim3(grid_for(n, kWPB, 16)), dim3(kBlock), 0, st, g->dag_off,
                       g->dag_adj, n, 2, kTcSmall, kTcMid, kTcMax, W.work, W.cls);
    GPM_LAUNCH_CHECK("k_root_work");
    const bool arcs = MODE == TC_ARCS;
    gpm_status rc = tc_class<kTcMax, 512, MODE>(
        g, W, RC_BIG, W.list_b, W.wpre_b, W.first_b, 2, g->tc_tau[2], g->tc_bpc[2],
        MODE == TC_LIST ? "k_tc_block<1024,list>" : (arcs ? "k_tc_block<1024,arcs>" : "k_tc_block<1024>"),
        res, te, em, st);
    if (rc) return rc;
    rc = tc_class<kTcMid, 256, MODE>(g, W, RC_MID, W.list_m, W.wpre_m, W.first_m, 1,
                                     g->tc_tau[1], g->tc_bpc[1],
                                     MODE == TC_LIST ? "k_tc_block<256,list>"
                                                     : (arcs ? "k_tc_block<256,arcs>" : "k_tc_block<256>"),
                                     res, te, em, st);
    if (rc) return rc;
    rc = tc_class<kTcSmall, 64, MODE>(g, W, RC_SMALL, W.list_s, W.wpre_s, W.first_s, 0,
                                      g->tc_tau[0], g->tc_bpc[0],
                                      MODE == TC_LIST ? "k_tc_block<64,list>"
                                                      : (arcs ? "k_tc_block<64,arcs>" : "k_tc_block<64>"),
                                      res, te, em, st);
    if (rc) return rc;
    constexpr int HM = MODE == TC_LIST ? HUB_LIST : (MODE == TC_ARCS ? HUB_ARCS : HUB_COUNT);
    return hub_launch<3, HM>(g, W, res, nullptr, nullptr, te, em, st);
}

gpm_status triangle_arc_counts(const gpm_graph *g, void *ws, uint64_t ws_bytes, uint32_t *te,
                               unsigned long long *tri, hipStream_t st) {
    CliqueWs W = clique_layout(g, 3, false, ws);
    if (W.bytes > ws_bytes) return fail(GPM_OUT_OF_MEMORY, "workspace smaller than required");
    return tc_launch<TC_ARCS>(g, W, tri, te, st);
}

gpm_status clique_run(const gpm_graph *g, int32_t k, bool list, void *ws, uint64_t ws_bytes,
                      unsigned long long *d_count, int32_t *d_buf, uint64_t cap,
                      unsigned long long *d_result, hipStream_t st) {
    CliqueWs W = clique_layout(g, k, list, ws);
    if (W.bytes > ws_bytes) return fail(GPM_OUT_OF_MEMORY, "workspace smaller than required");
    const int32_t n = g->n;
    unsigned long long *res = list ? d_result : W.result;
    GPM_HIP(fill_u32(res, 0, list ? 6 : 16, st));
    GPM_HIP(fill_u32(W.ctl, 0, 32, st));
    const bool generic = uses_generic(g, k, list);
    // listing through the triangle / local-graph kernels: slot counter in the
    // workspace, totals and checksum into d_result
    GPM_HIP(fill_u32(W.result, 0, 16, st));
    RowEmitter em{W.result + 6, d_buf, list ? cap : 0, 0, 0, 0};
    if (generic) {
        ListOut lo{d_buf, list ? cap : 0};
        int blocks = W.gen_waves / kWPB;
        if (list)
            hipLaunchKernelGGL(k_clique_generic<true>, dim3(blocks), dim3(kBlock), 0, st,
                               g->dag_off, g->dag_adj, n, k, std::max(1, g->max_out_degree),
                               W.gen_scratch, res, lo);
        else
            hipLaunchKernelGGL(k_clique_generic<false>, dim3(blocks), dim3(kBlock), 0, st,
                               g->dag_off, g->dag_adj, n, k, std::max(1, g->max_out_degree),
                               W.gen_scratch, res, lo);
        GPM_LAUNCH_CHECK("k_clique_generic");
        if (list) {
            hipLaunchKernelGGL(k_finish_listing, dim3(1), dim3(64), 0, st, res, cap);
            GPM_LAUNCH_CHECK("k_finish_listing");
        }
    } else if (k == 3) {
        gpm_status rc = list ? tc_launch<TC_LIST>(g, W, res, nullptr, st, em)
                             : tc_launch<TC_COUNT>(g, W, res, nullptr, st);
        if (rc) return rc;
    } else if (lg_disabled(k)) {
        // every root with out-degree >= k - 1 is a hub: one task per out-arc
        hipLaunchKernelGGL(k_root_work, dim3(grid_for(n, kWPB, 16)), dim3(kBlock), 0, st,
                           g->dag_off, g->dag_adj, n, k - 1, 0, 0, 0, W.work, W.cls);
        GPM_LAUNCH_CHECK("k_root_work");
        gpm_status rc;
        switch (k) {
        case 4: rc = list ? hub_launch<4, HUB_LIST>(g, W, res, nullptr, nullptr, nullptr, em, st, true)
                          : hub_launch<4, HUB_COUNT>(g, W, res, nullptr, nullptr, nullptr, em, st, true); break;
        case 5: rc = list ? hub_launch<5, HUB_LIST>(g, W, res, nullptr, nullptr, nullptr, em, st, true)
                          : hub_launch<5, HUB_COUNT>(g, W, res, nullptr, nullptr, nullptr, em, st, true); break;
        case 6: rc = hub_launch<6, HUB_COUNT>(g, W, res, nullptr, nullptr, nullptr, em, st, true); break;
        case 7: rc = hub_launch<7, HUB_COUNT>(g, W, res, nullptr, nullptr, nullptr, em, st, true); break;
        case 8: rc = hub_launch<8, HUB_COUNT>(g, W, res, nullptr, nullptr, nullptr, em, st, true); break;
        default: rc = hub_launch<9, HUB_COUNT>(g, W, res, nullptr, nullptr, nullptr, em, st, true); break;
        }
        if (rc) return rc;
    } else {
        hipLaunchKernelGGL(k_root_work, dim3(grid_for(n, kWPB, 16)), dim3(kBlock), 0, st,
                           g->dag_off, g->dag_adj, n, k - 1, 64, kMidMaxD, kTcMax, W.work, W.cls);
        GPM_LAUNCH_CHECK("k_root_work");
        {
            // three classes; each count lives in its own pos snapshot
            int32_t *cnt_s = (int32_t *)(W.ctl + 12), *cnt_m = (int32_t *)(W.ctl + 13),
                    *cnt_b = (int32_t *)(W.ctl + 14);
            GPM_HIP(build_class(g, W, RC_BIG, W.list_b, nullptr, st));
            GPM_HIP(hipMemcpyAsync(cnt_b, W.pos + n, 4, hipMemcpyDeviceToDevice, st));
            GPM_HIP(build_class(g, W, RC_MID, W.list_m, nullptr, st));
            GPM_HIP(hipMemcpyAsync(cnt_m, W.pos + n, 4, hipMemcpyDeviceToDevice, st));
            GPM_HIP(build_class(g, W, RC_SMALL, W.list_s, nullptr, st));
            GPM_HIP(hipMemcpyAsync(cnt_s, W.pos + n, 4, hipMemcpyDeviceToDevice, st));
            gpm_status rc;
            const RowEmitter *pem = list ? &em : nullptr;
            switch (k) {
            case 4: rc = launch_local<4>(g, W, cnt_s, cnt_m, cnt_b, res, nullptr, nullptr, st, pem); break;
            case 5: rc = launch_local<5>(g, W, cnt_s, cnt_m, cnt_b, res, nullptr, nullptr, st, pem); break;
            case 6: rc = launch_local<6>(g, W, cnt_s, cnt_m, cnt_b, res, nullptr, nullptr, st); break;
            case 7: rc = launch_local<7>(g, W, cnt_s, cnt_m, cnt_b, res, nullptr, nullptr, st); break;
            case 8: rc = launch_local<8>(g, W, cnt_s, cnt_m, cnt_b, res, nullptr, nullptr, st); break;
            default: rc = launch_local<9>(g, W, cnt_s, cnt_m, cnt_b, res, nullptr, nullptr, st); break;
            }
            if (rc) return rc;
        }
    }
    if (!list) GPM_HIP(hipMemcpyAsync(d_count, res, 8, hipMemcpyDeviceToDevice, st));
    if (list && !generic) {
        hipLaunchKernelGGL(k_finish_rows, dim3(1), dim3(64), 0, st, res, W.result + 6, cap);
        GPM_LAUNCH_CHECK("k_finish_rows");
    }
    return GPM_OK;
}

// Cliques of every size 3..kmax (kmax = 4 or 5) from one local-graph pass:
// the local graph of root u holds the triangles at u (its edges), the
// 4-cliques at u (its triangles) and the 5-cliques at u (its 4-cliques), so
// one build per root serves all sizes.  Roots need out-degree >= 2.
gpm_status clique_multi_workspace_bytes(const gpm_graph *g, int32_t kmax, uint64_t *bytes) {
    return clique_workspace_bytes(g, kmax, false, bytes);
}

gpm_status clique_multi_run(const gpm_graph *g, int32_t kmax, void *ws, uint64_t ws_bytes,
                            unsigned long long *d_counts, hipStream_t st) {
    if (kmax < 4 || kmax > 5) return fail(GPM_UNSUPPORTED, "kmax must be 4 or 5");
    CliqueWs W = clique_layout(g, kmax, false, ws);
    if (W.bytes > ws_bytes) return fail(GPM_OUT_OF_MEMORY, "workspace smaller than required");
    const int32_t n = g->n;
    unsigned long long *res = W.result;   // [0] k = kmax, [1] triangles, [2] 4-cliques (kmax 5)
    GPM_HIP(fill_u32(res, 0, 16, st));
    GPM_HIP(fill_u32(W.ctl, 0, 32, st));
    if (lg_disabled(kmax)) {
        // without local graphs: every root of out-degree >= 2 per arc
        hipLaunchKernelGGL(k_root_work, dim3(grid_for(n, kWPB, 16)), dim3(kBlock), 0, st,
                           g->dag_off, g->dag_adj, n, 2, 0, 0, 0, W.work, W.cls);
        GPM_LAUNCH_CHECK("k_root_work");
        gpm_status rc =
            kmax == 4 ? hub_launch<4, HUB_COUNT>(g, W, res, res + 1, nullptr, nullptr,
                                                 RowEmitter{}, st, true)
                      : hub_launch<5, HUB_COUNT>(g, W, res, res + 1, res + 2, nullptr,
                                                 RowEmitter{}, st, true);
        if (rc) return rc;
    } else {
        hipLaunchKernelGGL(k_root_work, dim3(grid_for(n, kWPB, 16)), dim3(kBlock), 0, st, g->dag_off,
                           g->dag_adj, n, 2, 64, kMidMaxD, kTcMax, W.work, W.cls);
        GPM_LAUNCH_CHECK("k_root_work");
        int32_t *cnt_s = (int32_t *)(W.ctl + 12), *cnt_m = (int32_t *)(W.ctl + 13),
                *cnt_b = (int32_t *)(W.ctl + 14);
        GPM_HIP(build_class(g, W, RC_BIG, W.list_b, nullptr, st));
        GPM_HIP(hipMemcpyAsync(cnt_b, W.pos + n, 4, hipMemcpyDeviceToDevice, st));
        GPM_HIP(build_class(g, W, RC_MID, W.list_m, nullptr, st));
        GPM_HIP(hipMemcpyAsync(cnt_m, W.pos + n, 4, hipMemcpyDeviceToDevice, st));
        GPM_HIP(build_class(g, W, RC_SMALL, W.list_s, nullptr, st));
        GPM_HIP(hipMemcpyAsync(cnt_s, W.pos + n, 4, hipMemcpyDeviceToDevice, st));
        gpm_status rc = kmax == 4
                            ? launch_local<4>(g, W, cnt_s, cnt_m, cnt_b, res, res + 1, nullptr, st)
                            : launch_local<5>(g, W, cnt_s, cnt_m, cnt_b, res, res + 1, res + 2, st);
        if (rc) return rc;
    }
    // d_counts = {triangles, 4-cliques[, 5-cliques]}
    GPM_HIP(hipMemcpyAsync(d_counts, res + 1, 8, hipMemcpyDeviceToDevice, st));
    if (kmax == 4) {
        GPM_HIP(hipMemcpyAsync(d_counts + 1, res, 8, hipMemcpyDeviceToDevice, st));
    } else {
        GPM_HIP(hipMemcpyAsync(d_counts + 1, res + 2, 8, hipMemcpyDeviceToDevice, st));
        GPM_HIP(hipMemcpyAsync(d_counts + 2, res, 8, hipMemcpyDeviceToDevice, st));
    }
    return GPM_OK;
}

}  // namespace gpm
