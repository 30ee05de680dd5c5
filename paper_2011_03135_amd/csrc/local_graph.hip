// Local-graph 4- and 5-clique counting for roots of out-degree 65..1024.
//
// For a root u of the degree-ordered DAG the local graph is the subgraph
// induced on N+(u), itself oriented (Section 5, search on a local graph; the
// local graph here is built once per root and kept as bit rows instead of
// being shrunk in place).  Row i holds, as a bit set over local indices, the
// out-neighbours of the i-th out-neighbour v_i that lie in N+(u).  Then
//   4-cliques rooted at u = sum over local edges (i, j) of |row_i & row_j|,
//   5-cliques rooted at u = sum over local edges (i, j), l in row_i & row_j
//                           of |row_i & row_j & row_l|.
// Rows are 64-bit words in LDS (at most 1024 x 16 words = 128 KiB of the
// 160 KiB a gfx950 workgroup may use).
//
// 4-cliques: one workgroup per root builds the rows and counts (counting
// costs about as much as building).
// 5-cliques: counting can cost far more than building on hub roots, so one
// kernel builds every root's rows once and stores them in HBM, and a second
// kernel splits each root into slices of its local edges (e = s mod S, S
// proportional to the root's local edge count times its row width); a slice
// copies the rows back into LDS and runs a per-lane work loop (fetch an
// edge, then step through its candidates one at a time) so skewed candidate
// sets do not stall a wave.
#include "gpm_internal.h"

#include <algorithm>

namespace gpm {

namespace {

constexpr int kMidMaxD = 256;
constexpr int kBigMaxD = 1024;
constexpr int kMidThreads = 256;
constexpr int kBigThreads = 1024;
// the big class's roots of out-degree 257..512 run at this bound: a third of
// the LDS, three workgroups per CU
constexpr int kHalfMaxD = 512;
constexpr int kHalfThreads = 512;
constexpr int kHalfBlocksPerCu = 3;
constexpr int32_t kMaxSlices = 1024;

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int last_le_i32(const int32_t *a, int n, int32_t x) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (a[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

// Position of the r-th set bit (0-based) of x; x must have more than r bits.
__device__ __forceinline__ int select_bit64(uint64_t x, int r) {
    int pos = 0;
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) {
        const int low = __popcll(x & ((1ull << s) - 1));
        if (r >= low) {
            r -= low;
            x >>= s;
            pos += s;
        }
    }
    return pos;
}

template <int NT>
struct Lds {
    int32_t s_sum[NT / kWave];
    uint32_t s_task, s_next;
    uint64_t s_tri;
};

// Hash table of a local-graph block: 4 slots per out-neighbour at the class
// bound (load factor <= 1/4); at the 1024 bound 2 (<= 1/4 up to half the
// bound, <= 1/2 at the bound), so its rows (128 KiB) and the table fit the
// 160 KiB of LDS.
template <int DMAX> struct LgHash {
    static constexpr int kSlots = DMAX >= 1024 ? 2 * DMAX : 4 * DMAX;
    static constexpr int kBits = DMAX >= 1024 ? 11 : (DMAX == 512 ? 11 : (DMAX == 256 ? 10 : 8));
    static_assert((1 << kBits) == kSlots, "slots must be a power of two");
};

// Builds the local graph of root u (d out-neighbours, W words per row) in
// LDS: row a gets bit b for every pair (v, w) of the root with v, w the
// out-neighbours of local indices a and b.  Local indices are positions in
// the out-list, or with RANK positions in the DAG's order, by (okey, id)
// (the graph's orientation key: degrees, or the core-value key); lidx, d
// entries, receives them.  That makes every row hold only bits above its
// own index.
// keys/vals/pre/offj are the root's staging area; ends with a barrier.
template <int DMAX, int NT, bool RANK>
__device__ void build_rows(const int32_t *__restrict__ off, const int32_t *__restrict__ okey,
                           const int32_t *__restrict__ dag_off,
                           const int32_t *__restrict__ dag_adj, int32_t u, int32_t d, int32_t W,
                           uint64_t *rows, int32_t *keys, int16_t *vals, int32_t *pre,
                           int32_t *offj, int16_t *lidx, int32_t *s_sum,
                           int32_t *verts = nullptr) {
    constexpr int PER = (DMAX + NT - 1) / NT;
    constexpr int NW = NT / kWave;
    constexpr int U = DMAX <= 256 ? 2 : 4;
    const int32_t s = dag_off[u];
    if (RANK) {
        // rank of each out-neighbour among the others, by (degree, id); the
        // row area is scratch for the keys until it is cleared below
        uint64_t *key = rows;
        for (int32_t i = threadIdx.x; i < d; i += NT) {
            const int32_t v = dag_adj[s + i];
            key[i] = ((uint64_t)(uint32_t)okey[v] << 32) | (uint32_t)v;
        }
        __syncthreads();
        for (int32_t i = threadIdx.x; i < d; i += NT) {
            const uint64_t k = key[i];
            int32_t c = 0;
            for (int32_t j = 0; j < d; j++) c += key[j] < k;
            lidx[i] = (int16_t)c;
        }
        __syncthreads();
    }
    const int32_t hb = min(lds_hash_bits(d), LgHash<DMAX>::kBits);
    for (int32_t i = threadIdx.x; i < (1 << hb); i += NT) keys[i] = -1;
    for (int32_t i = threadIdx.x; i < d * W; i += NT) rows[i] = 0ull;
    stage_root<NT, PER>(dag_off, dag_adj, s, d, keys, vals, hb, pre, offj, s_sum,
                        RANK ? lidx : nullptr, verts);
    const int32_t npairs = pre[d];
    const int32_t per_wave = ((npairs + NW - 1) / NW + U * kWave - 1) / (U * kWave) * (U * kWave);
    const int32_t qa = min(npairs, (int32_t)(threadIdx.x / kWave) * per_wave);
    const int32_t qz = min(npairs, qa + per_wave);
    walk_lookup<U>(pre, offj, dag_adj, d, qa, qz, keys, hb,
            [&](int32_t j, int32_t, int32_t w, int32_t slot) {
        if (slot >= 0) {
            const int32_t a = RANK ? (int32_t)lidx[j] : j;
            const int32_t b = vals[slot];
            atomicOr((unsigned long long *)&rows[a * W + (b >> 6)], 1ull << (b & 63));
        }
    });
    __syncthreads();
}

// pre[i] = number of local edges in rows 0..i-1; returns the total.
template <int DMAX, int NT>
__device__ int32_t row_prefix(const uint64_t *rows, int32_t d, int32_t W, int32_t *pre,
                              int32_t *s_sum) {
    constexpr int PER = (DMAX + NT - 1) / NT;
    int32_t pc[PER];
#pragma unroll
    for (int q = 0; q < PER; q++) {
        const int32_t i = threadIdx.x * PER + q;
        pc[q] = 0;
        if (i < d)
            for (int32_t w = 0; w < W; w++) pc[q] += __popcll(rows[i * W + w]);
    }
    block_prefix<NT, PER>(pc, d, pre, s_sum);
    return pre[d];
}

// Local edge number e -> (row i, column j).
__device__ __forceinline__ void edge_at(const uint64_t *rows, const int32_t *pre, int32_t d,
                                        int32_t W, int32_t e, int32_t &i, int32_t &j) {
    i = last_le_i32(pre, d + 1, e);
    int32_t rr = e - pre[i];
    const uint64_t *ri = rows + i * W;
    int32_t wj = 0;
    for (;; wj++) {
        const int pc = __popcll(ri[wj]);
        if (rr < pc) break;
        rr -= pc;
    }
    j = wj * 64 + select_bit64(ri[wj], rr);
}

__device__ __forceinline__ uint64_t uniform64(uint64_t x) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t wave_or64(uint64_t x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x |= __shfl_xor(x, o, 64);
    return uniform64(x);
}

// part + the sum over the columns b of word q listed in m (wave-uniform) of
// [bit b of X[q]] * sum over w >= q of popc(X[w] & row_b[w]).  The halves of
// the word are walked one after the other, so the lane's bit test is one
// bit-field extract of a 32-bit register and its product with the count one
// 24-bit multiply-add; row_b is a broadcast LDS read.
template <int W>
__device__ __forceinline__ uint32_t pair_sweep(const uint64_t *rows, const uint64_t (&X)[W], int q,
                                               uint64_t m, uint32_t part) {
#pragma unroll
    for (int h = 0; h < 2; h++) {
        const uint32_t x = (uint32_t)(X[q] >> (32 * h));
        uint32_t mh = (uint32_t)(m >> (32 * h));
        while (mh) {
            const int bp = __builtin_ctz(mh);
            mh &= mh - 1u;
            const uint64_t *yb = rows + (q * kWave + h * 32 + bp) * W;
            uint32_t sc = 0;
#pragma unroll
            for (int w = q; w < W; w++) sc += (uint32_t)__popcll(X[w] & yb[w]);
            // written as instructions: the compiler would otherwise turn the
            // 0/1 product into a compare and a select
            uint32_t bit, np;
            asm("v_bfe_u32 %0, %1, %2, 1" : "=v"(bit) : "v"(x), "s"(bp));
            asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(np) : "v"(bit), "v"(sc), "v"(part));
            part = np;
        }
    }
    return part;
}

// Triangles of a local graph in degree order (d vertices, W words per row,
// every row holding only bits above its own index): the sum over local
// edges a -> b of |row_a & row_b|.  The work is cut into pieces (t, q): rows
// 64t..64t+63 (one per lane, in registers) against the columns b of word q
// (q >= t).  b runs over the union of the 64 rows' bits in word q in a
// wave-uniform loop, so row_b is a broadcast LDS read, and the AND +
// population count covers the words from q up.  Pieces go round robin to the
// workgroup's waves in order of q, i.e. from the costliest (W - q words per
// column) down.  Returns the calling lane's share.
template <int W>
__device__ uint64_t local_tri(const uint64_t *rows, int32_t d, int wib, int nw) {
    const int lane = lane_id();
    constexpr int kPieces = W * (W + 1) / 2;
    uint64_t acc = 0;
    for (int p = wib; p < kPieces; p += nw) {
        int q = 0;
        while ((q + 1) * (q + 2) / 2 <= p) q++;
        const int t = p - q * (q + 1) / 2;
        const int32_t a = t * kWave + lane;
        if (t * kWave >= d) continue;
        uint32_t part = 0;
#pragma unroll
        for (int qq = 0; qq < W; qq++) {
            if (qq != q) continue;
            uint64_t X[W];
#pragma unroll
            for (int w = qq; w < W; w++) X[w] = a < d ? rows[a * W + w] : 0ull;
            part = pair_sweep<W>(rows, X, qq, wave_or64(X[qq]), part);
        }
        acc += part;
    }
    return acc;
}

template <int WLO, int WHI>
__device__ __forceinline__ uint64_t local_tri_dispatch(int32_t W, const uint64_t *rows, int32_t d,
                                                       int wib, int nw) {
    if constexpr (WLO > WHI) {
        return 0;
    } else {
        if (W == WLO) return local_tri<WLO>(rows, d, wib, nw);
        return local_tri_dispatch<WLO + 1, WHI>(W, rows, d, wib, nw);
    }
}

// 4-cliques: workgroup per root (atomic cursor over the class list; roots of
// out-degree <= dlo are left to another launch); the root's 4-cliques are the
// triangles of its local graph.  RANK puts the local graph in degree order
// and counts its triangles with local_tri, else they are counted per local
// edge.  With LIST every 4-clique (u, v_i, v_j, v_x) is emitted instead.
template <int DMAX, int NT, bool LIST, bool RANK>
__global__ void __launch_bounds__(NT, DMAX == kHalfMaxD ? 6 : 1) k_lg4(const int32_t *__restrict__ off,
                                            const int32_t *__restrict__ okey,
                                            const int32_t *__restrict__ dag_off,
                                            const int32_t *__restrict__ dag_adj,
                                            const int32_t *__restrict__ roots,
                                            const int32_t *__restrict__ nroots_p, int32_t dlo,
                                            uint32_t *cursor, unsigned long long *result,
                                            unsigned long long *res3, RowEmitter em) {
    __shared__ uint64_t rows[DMAX * (DMAX / 64)];
    __shared__ __align__(16) int32_t keys[LgHash<DMAX>::kSlots];
    __shared__ int16_t vals[LgHash<DMAX>::kSlots];
    __shared__ int32_t offj[DMAX], pre[DMAX + 1];
    __shared__ int32_t verts[LIST ? DMAX : 1];
    __shared__ int16_t lidx[RANK ? DMAX : 1];
    __shared__ Lds<NT> sh;
    const int tid = threadIdx.x;
    const int32_t nroots = *nroots_p;
    uint64_t acc = 0;
    for (;;) {
        if (tid == 0) sh.s_task = atomicAdd(cursor, 1u);
        __syncthreads();
        const int32_t r = (int32_t)sh.s_task;
        __syncthreads();
        if (r >= nroots) break;
        const int32_t u = roots[r];
        const int32_t d = dag_off[u + 1] - dag_off[u], W = (d + 63) >> 6;
        if (d <= dlo || d > DMAX) continue;
        build_rows<DMAX, NT, RANK>(off, okey, dag_off, dag_adj, u, d, W, rows, keys, vals, pre, offj,
                                   RANK ? lidx : nullptr, sh.s_sum, LIST ? verts : nullptr);
        const int32_t ne = row_prefix<DMAX, NT>(rows, d, W, pre, sh.s_sum);
        if (res3 && tid == 0 && ne) atomicAdd(res3, (unsigned long long)ne);   // triangles at u
        if constexpr (LIST || !RANK) {
            for (int32_t e = tid; e < ne; e += NT) {
                int32_t i, j;
                edge_at(rows, pre, d, W, e, i, j);
                const uint64_t *ri = rows + i * W, *rj = rows + j * W;
                if constexpr (LIST) {
                    for (int32_t w = 0; w < W; w++) {
                        uint64_t m = ri[w] & rj[w];
                        while (m) {
                            const int32_t x = w * 64 + __builtin_ctzll(m);
                            m &= m - 1ull;
                            const int32_t q[4] = {u, verts[i], verts[j], verts[x]};
                            emit_vertices<4>(em, q);
                        }
                    }
                } else {
                    for (int32_t w = 0; w < W; w++) acc += __popcll(ri[w] & rj[w]);
                }
            }
        } else if (ne) {
            acc += local_tri_dispatch<1, DMAX / kWave>(W, rows, d, tid / kWave, NT / kWave);
        }
        __syncthreads();
    }
    if (LIST) {
        row_emitter_flush(em, result);
        return;
    }
    acc = wave_sum(acc);
    if (lane_id() == 0 && acc) atomicAdd(result, (unsigned long long)acc);
}

// 5-cliques, step 1: rows of every root (local indices in degree order) to
// HBM, and local triangle counts for slicing.
template <int DMAX, int NT>
__global__ void __launch_bounds__(NT, DMAX == kHalfMaxD ? 6 : 1) k_lg_build(const int32_t *__restrict__ off,
                                                 const int32_t *__restrict__ okey,
                                                 const int32_t *__restrict__ dag_off,
                                                 const int32_t *__restrict__ dag_adj,
                                                 const int32_t *__restrict__ roots,
                                                 const int32_t *__restrict__ nroots_p, int32_t dlo,
                                                 uint32_t *cursor, const int64_t *__restrict__ rowoff,
                                                 uint64_t *grows, int32_t *slices,
                                                 unsigned long long *units,
                                                 unsigned long long *res3,
                                                 unsigned long long *res4, uint64_t slice5) {
    __shared__ uint64_t rows[DMAX * (DMAX / 64)];
    __shared__ __align__(16) int32_t keys[LgHash<DMAX>::kSlots];
    __shared__ int16_t vals[LgHash<DMAX>::kSlots];
    __shared__ int16_t lidx[DMAX];
    __shared__ int32_t offj[DMAX], pre[DMAX + 1];
    __shared__ int32_t verts[DMAX];
    __shared__ Lds<NT> sh;
    const int tid = threadIdx.x;
    const int32_t nroots = *nroots_p;
    if (tid == 0) sh.s_tri = 0;
    for (;;) {
        if (tid == 0) sh.s_task = atomicAdd(cursor, 1u);
        __syncthreads();
        const int32_t r = (int32_t)sh.s_task;
        __syncthreads();
        if (r >= nroots) break;
        const int32_t u = roots[r];
        const int32_t d = dag_off[u + 1] - dag_off[u], W = (d + 63) >> 6;
        if (d <= dlo || d > DMAX) continue;
        build_rows<DMAX, NT, true>(off, okey, dag_off, dag_adj, u, d, W, rows, keys, vals, pre, offj,
                                   lidx, sh.s_sum, verts);
        uint64_t *dst = grows + rowoff[r];
        for (int32_t i = tid; i < d * W; i += NT) dst[i] = rows[i];
        // then the out-neighbours in local (degree) order, for listings
        int32_t *dverts = reinterpret_cast<int32_t *>(dst + d * W);
        for (int32_t i = tid; i < d; i += NT) dverts[i] = verts[i];
        const int32_t ne = row_prefix<DMAX, NT>(rows, d, W, pre, sh.s_sum);
        if (res3 && tid == 0 && ne) atomicAdd(res3, (unsigned long long)ne);   // triangles at u
        // local triangles (the 4-cliques at u): the 5-clique work
        uint64_t tri = ne ? local_tri_dispatch<1, DMAX / kWave>(W, rows, d, tid / kWave, NT / kWave)
                          : 0;
        tri = wave_sum(tri);
        if (lane_id() == 0 && tri) atomicAdd((unsigned long long *)&sh.s_tri, (unsigned long long)tri);
        __syncthreads();
        if (tid == 0) {
            // slices over local vertices: about slice5 local triangles each
            // (per graph, gpm_graph::lg5_slice), at least 8 local vertices each
            const uint64_t s_work = 1 + sh.s_tri / slice5;
            const uint64_t s_cap = (uint64_t)(d / 8 + 1);
            slices[r] = (int32_t)std::min<uint64_t>(kMaxSlices, std::min(s_work, s_cap));
            if (sh.s_tri) atomicAdd(units, (unsigned long long)sh.s_tri);
            if (sh.s_tri && res4) atomicAdd(res4, (unsigned long long)sh.s_tri);
            sh.s_tri = 0;
        }
        __syncthreads();
    }
}

// Storage words of every class root (d * W row words and d vertex ids), for
// the row storage prefix.
__global__ void k_lg_words(const int32_t *dag_off, const int32_t *roots, const int32_t *nroots_p,
                           int32_t *words) {
    const int32_t nroots = *nroots_p;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < nroots; i += stride) {
        const int32_t u = roots[i], d = dag_off[u + 1] - dag_off[u];
        words[i] = d * ((d + 63) >> 6) + (d + 1) / 2;   // rows, then d int32 vertex ids
    }
}

// 5-cliques, step 2: task (root, slice); rows come back from HBM into LDS.
// For local vertex i with out-row R (members p_0 < ... < p_{c-1}), the
// 5-cliques {u, v_i, ...} are the triangles a < b < x of the local DAG
// inside R: the sum over members a < b of [a -> b] * |row_a & R & row_b|.
// Lanes own a (64 members at a time, row_a & R in registers); b runs over
// R's members in a wave-uniform loop, so row_b is a broadcast LDS read, and
// the AND + population count runs over the words from b's word up (a row
// only holds bits above its own vertex).  Local graphs of hub roots are
// dense, so testing every pair costs little more than following edges and
// keeps all 64 lanes busy.
// LDS is dynamic: rows (dmax x ceil(dmax/64) words for the class's largest
// out-degree), then per wave a member list of DMAX int16.

template <int W>
__device__ uint64_t lg5_vertex(const uint64_t *rows, const uint64_t *ri, int32_t c, int16_t *mem) {
    const int lane = lane_id();
    uint64_t R[W];
#pragma unroll
    for (int q = 0; q < W; q++) R[q] = uniform64(ri[q]);
    int32_t base = 0;
#pragma unroll
    for (int q = 0; q < W; q++) {
        if ((R[q] >> lane) & 1ull) mem[base + lanes_below(R[q])] = (int16_t)(q * 64 + lane);
        base += __popcll(R[q]);
    }
    wave_sync();
    uint64_t acc = 0;
    for (int32_t a0 = 0; a0 < c; a0 += kWave) {
        const int32_t a = a0 + lane;
        uint64_t X[W];
        if (a < c) {
            const uint64_t *ra = rows + (int32_t)mem[a] * W;
#pragma unroll
            for (int q = 0; q < W; q++) X[q] = ra[q] & R[q];
        } else {
#pragma unroll
            for (int q = 0; q < W; q++) X[q] = 0ull;
        }
        const int32_t p0 = __builtin_amdgcn_readfirstlane((int32_t)mem[a0]);
        const int32_t q0 = p0 >> 6;
        uint32_t part = 0;
#pragma unroll
        for (int q = 0; q < W; q++) {
            if (q < q0) continue;
            uint64_t m = R[q];
            if (q == q0) m &= ~((2ull << (p0 & 63)) - 1ull);   // members above p0
            part = pair_sweep<W>(rows, X, q, m, part);
        }
        acc += part;
    }
    wave_sync();
    return acc;
}

// Listing form of lg5_vertex: emits every 5-clique {u, v_i, a, b, x} with
// a < b < x a triangle inside R (vertex ids from verts, the out-neighbours
// in local order).
template <int W>
__device__ void lg5_list(const uint64_t *rows, const uint64_t *ri, int32_t c, int16_t *mem,
                         const int32_t *verts, int32_t u, int32_t vi, RowEmitter &em) {
    const int lane = lane_id();
    uint64_t R[W];
#pragma unroll
    for (int q = 0; q < W; q++) R[q] = uniform64(ri[q]);
    int32_t base = 0;
#pragma unroll
    for (int q = 0; q < W; q++) {
        if ((R[q] >> lane) & 1ull) mem[base + lanes_below(R[q])] = (int16_t)(q * 64 + lane);
        base += __popcll(R[q]);
    }
    wave_sync();
    for (int32_t a0 = 0; a0 < c; a0 += kWave) {
        const int32_t a = a0 + lane;
        uint64_t X[W];
        int32_t pa = 0;
        if (a < c) {
            pa = mem[a];
            const uint64_t *ra = rows + pa * W;
#pragma unroll
            for (int q = 0; q < W; q++) X[q] = ra[q] & R[q];
        } else {
#pragma unroll
            for (int q = 0; q < W; q++) X[q] = 0ull;
        }
        const int32_t p0 = __builtin_amdgcn_readfirstlane((int32_t)mem[a0]);
        const int32_t q0 = p0 >> 6;
#pragma unroll
        for (int q = 0; q < W; q++) {
            if (q < q0) continue;
            uint64_t m = R[q];
            if (q == q0) m &= ~((2ull << (p0 & 63)) - 1ull);
            while (m) {
                const int bp = __builtin_ctzll(m);
                m &= m - 1ull;
                const int32_t pb = q * 64 + bp;
                if ((X[q] >> bp) & 1ull) {
                    const uint64_t *yb = rows + pb * W;
#pragma unroll
                    for (int w = q; w < W; w++) {
                        uint64_t mm = X[w] & yb[w];
                        while (mm) {
                            const int32_t x = w * 64 + __builtin_ctzll(mm);
                            mm &= mm - 1ull;
                            const int32_t clq[5] = {u, vi, verts[pa], verts[pb], verts[x]};
                            emit_vertices<5>(em, clq);
                        }
                    }
                }
            }
        }
    }
    wave_sync();
}

template <int WLO, int WHI>
__device__ __forceinline__ void lg5_list_dispatch(int32_t W, const uint64_t *rows,
                                                  const uint64_t *ri, int32_t c, int16_t *mem,
                                                  const int32_t *verts, int32_t u, int32_t vi,
                                                  RowEmitter &em) {
    if constexpr (WLO <= WHI) {
        if (W == WLO) lg5_list<WLO>(rows, ri, c, mem, verts, u, vi, em);
        else lg5_list_dispatch<WLO + 1, WHI>(W, rows, ri, c, mem, verts, u, vi, em);
    }
}

// (e + 3)-cliques of the local DAG inside the set S (W words, c >= 3
// members): for e = 0 the triangles inside S; for e > 0 the sum over members
// v of S of the (e + 2)-cliques inside S & row_v (rows hold only bits above
// their own index, so each clique is found once, from its lowest member).
// The descent is wave-uniform and iterative: level l keeps its set and the
// members still to visit in the wave's stack area (2 W words per level,
// e + 1 levels), the deepest child set in the last slot.
template <int W>
__device__ uint64_t lgk_set(const uint64_t *rows, const uint64_t *S, int32_t c, int32_t e,
                            int16_t *mem, uint64_t *stack) {
    if (e == 0) return lg5_vertex<W>(rows, S, c, mem);
    uint64_t acc = 0;
#pragma unroll
    for (int q = 0; q < W; q++) {
        const uint64_t x = uniform64(S[q]);
        stack[q] = x;
        stack[W + q] = x;
    }
    wave_sync();
    int32_t lvl = 0;
    while (lvl >= 0) {
        uint64_t *set = stack + lvl * 2 * W, *rem = set + W;
        int32_t v = -1;
#pragma unroll
        for (int q = 0; q < W; q++) {
            const uint64_t r = uniform64(rem[q]);
            if (v < 0 && r) {
                v = q * 64 + __builtin_ctzll(r);
                rem[q] = r & (r - 1ull);
            }
        }
        wave_sync();
        if (v < 0) {
            lvl--;
            continue;
        }
        const uint64_t *rv = rows + v * W;
        uint64_t *child = stack + (lvl + 1) * 2 * W;
        int32_t cnt = 0;
#pragma unroll
        for (int q = 0; q < W; q++) {
            const uint64_t x = uniform64(set[q]) & uniform64(rv[q]);
            child[q] = x;
            child[W + q] = x;
            cnt += __popcll(x);
        }
        wave_sync();
        if (lvl + 1 == e) {
            if (cnt >= 3) acc += lg5_vertex<W>(rows, child, cnt, mem);
        } else if (cnt >= e - lvl + 2) {
            lvl++;
        }
    }
    return acc;
}

template <int WLO, int WHI>
__device__ __forceinline__ uint64_t lg5_dispatch(int32_t W, const uint64_t *rows, const uint64_t *ri,
                                                 int32_t c, int32_t e, int16_t *mem,
                                                 uint64_t *stack) {
    if constexpr (WLO > WHI) {
        return 0;
    } else {
        if (W == WLO) return lgk_set<WLO>(rows, ri, c, e, mem, stack);
        return lg5_dispatch<WLO + 1, WHI>(W, rows, ri, c, e, mem, stack);
    }
}

template <int DMAX, bool LIST>
__global__ void __launch_bounds__(1024) k_lg5(const int32_t *__restrict__ dag_off,
                                              const int32_t *__restrict__ roots,
                                              const int32_t *__restrict__ toff,
                                              const int32_t *__restrict__ nroots_p,
                                              const int64_t *__restrict__ rowoff,
                                              const uint64_t *__restrict__ grows,
                                              int32_t rows_words, int32_t extra,
                                              uint32_t *cursor, unsigned long long *result,
                                              RowEmitter em) {
    // row widths of the class: out-degrees (DMAX/4, DMAX]
    constexpr int WLO = DMAX / 256 + 1, WHI = DMAX / 64;
    extern __shared__ uint64_t dyn[];
    uint64_t *rows = dyn;
    __shared__ Lds<1024> sh;
    const int tid = threadIdx.x, lane = lane_id(), wib = tid / kWave;
    const int NT = blockDim.x;
    // then the out-neighbours in local order (listing), then per wave: member
    // list (DMAX int16) and the descent stack
    int32_t *verts = reinterpret_cast<int32_t *>(dyn + rows_words);
    uint8_t *wave_area = reinterpret_cast<uint8_t *>(verts + DMAX) +
                         (size_t)wib * (DMAX * 2 + (size_t)(extra + 1) * 2 * (DMAX / 64) * 8);
    int16_t *mem = reinterpret_cast<int16_t *>(wave_area);
    uint64_t *stack = reinterpret_cast<uint64_t *>(wave_area + DMAX * 2);
    const int32_t nroots = *nroots_p;
    const int32_t ntasks = toff[nroots];
    uint64_t acc = 0;
    for (;;) {
        if (tid == 0) sh.s_task = atomicAdd(cursor, 1u);
        __syncthreads();
        const int32_t t = (int32_t)sh.s_task;
        __syncthreads();
        if (t >= ntasks) break;
        const int32_t r = last_le_i32(toff, nroots + 1, t);
        const int32_t slice = t - toff[r], S = toff[r + 1] - toff[r];
        const int32_t u = roots[r];
        const int32_t d = dag_off[u + 1] - dag_off[u], W = (d + 63) >> 6;
        const uint64_t *src = grows + rowoff[r];
        for (int32_t i = tid; i < d * W; i += NT) rows[i] = src[i];
        if (LIST) {
            const int32_t *sv = reinterpret_cast<const int32_t *>(src + d * W);
            for (int32_t i = tid; i < d; i += NT) verts[i] = sv[i];
        }
        if (tid == 0) sh.s_next = 0;
        __syncthreads();
        // waves take the slice's local vertices i = slice + S * c
        for (;;) {
            uint32_t c = 0;
            if (lane == 0) c = atomicAdd(&sh.s_next, 1u);
            c = __shfl(c, 0, 64);
            const int32_t i = slice + S * (int32_t)c;
            if (i >= d) break;
            const uint64_t *ri = rows + i * W;
            int32_t cnt = 0;
            for (int32_t w = 0; w < W; w++) cnt += __popcll(ri[w]);
            if (cnt < 3 + extra) continue;
            if constexpr (LIST)
                lg5_list_dispatch<WLO, WHI>(W, rows, ri, cnt, mem, verts, u, verts[i], em);
            else
                acc += lg5_dispatch<WLO, WHI>(W, rows, ri, cnt, extra, mem, stack);
        }
        __syncthreads();
    }
    if (LIST) {
        row_emitter_flush(em, result);
        return;
    }
    acc = wave_sum(acc);
    if (lane == 0 && acc) atomicAdd(result, (unsigned long long)acc);
}

// k >= 5 for roots of out-degree 65..256, build and count in one kernel: a
// workgroup builds the root's local graph in LDS (degree order), adds its
// local edges (triangles at u) to res3 and its local triangles (4-cliques at
// u) to res4 when asked, then its waves take the level-1 vertices and count
// (or list) as k_lg5 does.  The local graphs are small, so no slicing and no
// trip through HBM.
template <int DMAX, int NT, bool LIST>
__global__ void __launch_bounds__(NT) k_lg5_mid(const int32_t *__restrict__ off,
                                                const int32_t *__restrict__ okey,
                                                const int32_t *__restrict__ dag_off,
                                                const int32_t *__restrict__ dag_adj,
                                                const int32_t *__restrict__ roots,
                                                const int32_t *__restrict__ nroots_p,
                                                int32_t extra, uint32_t *cursor,
                                                unsigned long long *result,
                                                unsigned long long *res3,
                                                unsigned long long *res4, RowEmitter em) {
    constexpr int NW = NT / kWave;
    constexpr int WMAX = DMAX / 64;
    constexpr int WLO = 2, WHI = WMAX;   // out-degrees 65..DMAX
    constexpr int kMaxExtra = 4;         // k <= 9
    __shared__ uint64_t rows[DMAX * WMAX];
    __shared__ __align__(16) int32_t keys[LgHash<DMAX>::kSlots];
    __shared__ int16_t vals[LgHash<DMAX>::kSlots];
    __shared__ int16_t lidx[DMAX];
    __shared__ int32_t offj[DMAX], pre[DMAX + 1];
    __shared__ int32_t verts[DMAX];
    __shared__ int16_t s_mem[NW][DMAX];
    __shared__ uint64_t s_stack[NW][(kMaxExtra + 1) * 2 * WMAX];
    __shared__ Lds<NT> sh;
    const int tid = threadIdx.x, lane = lane_id(), wib = tid / kWave;
    const int32_t nroots = *nroots_p;
    uint64_t acc = 0, acc3 = 0, acc4 = 0;
    for (;;) {
        if (tid == 0) sh.s_task = atomicAdd(cursor, 1u);
        __syncthreads();
        const int32_t r = (int32_t)sh.s_task;
        __syncthreads();
        if (r >= nroots) break;
        const int32_t u = roots[r];
        const int32_t d = dag_off[u + 1] - dag_off[u], W = (d + 63) >> 6;
        build_rows<DMAX, NT, true>(off, okey, dag_off, dag_adj, u, d, W, rows, keys, vals, pre, offj,
                                   lidx, sh.s_sum, verts);
        if (res3 || res4) {
            const int32_t ne = row_prefix<DMAX, NT>(rows, d, W, pre, sh.s_sum);
            if (tid == 0) acc3 += ne;
            if (res4)
                for (int32_t e = tid; e < ne; e += NT) {
                    int32_t i, j;
                    edge_at(rows, pre, d, W, e, i, j);
                    const uint64_t *ri = rows + i * W, *rj = rows + j * W;
                    for (int32_t w = 0; w < W; w++) acc4 += __popcll(ri[w] & rj[w]);
                }
        }
        for (int32_t i = wib; i < d; i += NW) {
            const uint64_t *ri = rows + i * W;
            int32_t cnt = 0;
            for (int32_t w = 0; w < W; w++) cnt += __popcll(ri[w]);
            if (cnt < 3 + extra) continue;
            if constexpr (LIST)
                lg5_list_dispatch<WLO, WHI>(W, rows, ri, cnt, s_mem[wib], verts, u, verts[i], em);
            else
                acc += lg5_dispatch<WLO, WHI>(W, rows, ri, cnt, extra, s_mem[wib], s_stack[wib]);
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
    if (res4) {
        acc4 = wave_sum(acc4);
        if (lane == 0 && acc4) atomicAdd(res4, (unsigned long long)acc4);
    }
}

struct LgWs {
    uint32_t *ctl;                 // cursors
    unsigned long long *units;     // per class: local triangles (5-cliques' work)
    int32_t *words, *slices, *toff_b;
    int64_t *rowoff_b, *scan_tmp;
    uint64_t *rows_b;
    uint64_t bytes;
};

LgWs lg_layout(const gpm_graph *g, int32_t k, void *base) {
    LgWs L{};
    Carve c(base, ~0ull);
    const uint64_t n1 = (uint64_t)g->n + 1;
    L.ctl = c.take<uint32_t>(16);
    L.units = c.take<unsigned long long>(4);
    if (k >= 5) {
        L.words = c.take<int32_t>(n1);
        L.slices = c.take<int32_t>(n1);
        L.toff_b = c.take<int32_t>(n1);
        L.rowoff_b = c.take<int64_t>(n1);
        L.scan_tmp = c.take<int64_t>(scan_tmp_words(n1));
        // rows and vertex ids of all roots with out-degree in (256, 1024]: sum of
        // d * ceil(d / 64) + ceil(d / 2) <= m * (ceil(max_out / 64) + 1) words
        const uint64_t wmax = (uint64_t)(std::max(g->max_out_degree, 1) + 63) / 64 + 1;
        const uint64_t words = (uint64_t)std::max<int64_t>(g->m, 1) * wmax + (uint64_t)g->n;
        L.rows_b = c.take<uint64_t>(words);
    }
    L.bytes = c.used;
    return L;
}

unsigned grid_for(int64_t items, int per_block, int cap_per_cu) {
    int64_t b = (items + per_block - 1) / per_block;
    int64_t cap = (int64_t)cu_count() * cap_per_cu;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

template <int DMAX, int NT>
gpm_status lg5_class(const gpm_graph *g, int32_t k, LgWs &L, const int32_t *list,
                     const int32_t *cnt,
                     int64_t *rowoff, uint64_t *rows, unsigned long long *units, int32_t *toff,
                     uint32_t *cursors, unsigned long long *res, unsigned long long *res3,
                     unsigned long long *res4, const RowEmitter *em, hipStream_t st,
                     const char *nb, const char *nc) {
    const int32_t n = g->n;
    GPM_HIP(fill_u32(L.words, 0, (uint64_t)n + 1, st));
    hipLaunchKernelGGL(k_lg_words, dim3(grid_for(n, 256, 8)), dim3(256), 0, st, g->dag_off, list,
                       cnt, L.words);
    GPM_LAUNCH_CHECK("k_lg_words");
    GPM_HIP(exclusive_scan_i64(L.words, rowoff, (uint64_t)n, L.scan_tmp, st));
    GPM_HIP(fill_u32(L.slices, 0, (uint64_t)n + 1, st));
    if constexpr (DMAX > kHalfMaxD) {
        // roots of out-degree up to kHalfMaxD at the smaller bound, the rest here
        Span sp("k_lg_build<512>", st);
        hipLaunchKernelGGL((k_lg_build<kHalfMaxD, kHalfThreads>),
                           dim3((unsigned)cu_count() * kHalfBlocksPerCu), dim3(kHalfThreads), 0,
                           st, g->off, g->okey, g->dag_off, g->dag_adj, list, cnt, kMidMaxD, cursors + 2,
                           rowoff, rows, L.slices, units, res3, res4, (uint64_t)g->lg5_slice);
    }
    GPM_LAUNCH_CHECK("k_lg_build<512>");
    {
        Span sp(nb, st);
        hipLaunchKernelGGL((k_lg_build<DMAX, NT>), dim3((unsigned)cu_count() * (NT <= 256 ? 8 : 1)),
                           dim3(NT), 0, st, g->off, g->okey, g->dag_off, g->dag_adj, list, cnt,
                           DMAX > kHalfMaxD ? kHalfMaxD : 0, cursors + 0, rowoff, rows, L.slices,
                           units, res3, res4, (uint64_t)g->lg5_slice);
    }
    GPM_LAUNCH_CHECK("k_lg_build");
    GPM_HIP(exclusive_scan_i32(L.slices, toff, (uint64_t)n, L.scan_tmp, st));
    {
        // LDS: rows of the class's largest local graph, then per-wave member
        // lists; as many waves as fit in 160 KiB (at most 16)
        const int32_t dmax = std::min<int32_t>(DMAX, std::max(g->max_out_degree, 1));
        const int32_t rows_words = dmax * ((dmax + 63) / 64);
        const int64_t lds_cap = 160 * 1024 - 1024;
        const int32_t extra = k - 5;
        const int64_t per_wave = (int64_t)DMAX * 2 + (int64_t)(extra + 1) * 2 * (DMAX / 64) * 8;
        // rows, the local vertex ids, then the per-wave areas
        const int64_t fixed = (int64_t)rows_words * 8 + (int64_t)DMAX * 4;
        int waves = (int)std::min<int64_t>(DMAX <= 256 ? 4 : 16, (lds_cap - fixed) / per_wave);
        if (waves < 1) return fail(GPM_DEVICE_ERROR, "local graph does not fit in LDS");
        const size_t shmem = (size_t)fixed + (size_t)waves * per_wave;
        Span sp(nc, st);
        const dim3 grid((unsigned)cu_count() * (DMAX <= 256 ? 4 : 1));
        if (em)
            hipLaunchKernelGGL((k_lg5<DMAX, true>), grid, dim3(waves * kWave), shmem, st,
                               g->dag_off, list, toff, cnt, rowoff, (const uint64_t *)rows,
                               rows_words, extra, cursors + 1, res, *em);
        else
            hipLaunchKernelGGL((k_lg5<DMAX, false>), grid, dim3(waves * kWave), shmem, st,
                               g->dag_off, list, toff, cnt, rowoff, (const uint64_t *)rows,
                               rows_words, extra, cursors + 1, res, RowEmitter{});
        span_units(units, st);
    }
    GPM_LAUNCH_CHECK("k_lg5");
    return GPM_OK;
}

}  // namespace

gpm_status lg_workspace_bytes(const gpm_graph *g, int32_t k, uint64_t *bytes) {
    *bytes = lg_layout(g, k, nullptr).bytes;
    return GPM_OK;
}

// Counts k-cliques (k = 4..9) rooted at the two workgroup classes: list_m
// (out-degree 65..256) and list_b (257..1024), device counts cnt_m, cnt_b,
// into *res.  res3 / res4 (may be null) also receive the triangles and (for
// k = 5) the 4-cliques rooted at the same roots.
gpm_status lg_cliques(const gpm_graph *g, int32_t k, const int32_t *list_m, const int32_t *cnt_m,
                      const int32_t *list_b, const int32_t *cnt_b, void *ws, uint64_t ws_bytes,
                      unsigned long long *res, unsigned long long *res3,
                      unsigned long long *res4, const RowEmitter *em, hipStream_t st) {
    LgWs L = lg_layout(g, k, ws);
    if (L.bytes > ws_bytes) return fail(GPM_OUT_OF_MEMORY, "local-graph workspace too small");
    GPM_HIP(fill_u32(L.ctl, 0, 16, st));
    GPM_HIP(fill_u32(L.units, 0, 8, st));
    if (k == 4) {
        const RowEmitter none{};
        {
            Span sp("k_lg4<1024>", st);
            if (em)
                hipLaunchKernelGGL((k_lg4<kBigMaxD, kBigThreads, true, true>),
                                   dim3((unsigned)cu_count()), dim3(kBigThreads), 0, st, g->off,
                                   g->okey, g->dag_off, g->dag_adj, list_b, cnt_b, kHalfMaxD,
                                   L.ctl + 0, res, res3, *em);
            else
                hipLaunchKernelGGL((k_lg4<kBigMaxD, kBigThreads, false, true>),
                                   dim3((unsigned)cu_count()), dim3(kBigThreads), 0, st, g->off,
                                   g->okey, g->dag_off, g->dag_adj, list_b, cnt_b, kHalfMaxD,
                                   L.ctl + 0, res, res3, none);
        }
        GPM_LAUNCH_CHECK("k_lg4<1024>");
        {
            Span sp("k_lg4<512>", st);
            const dim3 grid((unsigned)cu_count() * kHalfBlocksPerCu);
            if (em)
                hipLaunchKernelGGL((k_lg4<kHalfMaxD, kHalfThreads, true, true>), grid,
                                   dim3(kHalfThreads), 0, st, g->off, g->okey, g->dag_off, g->dag_adj,
                                   list_b, cnt_b, kMidMaxD, L.ctl + 2, res, res3, *em);
            else
                hipLaunchKernelGGL((k_lg4<kHalfMaxD, kHalfThreads, false, true>), grid,
                                   dim3(kHalfThreads), 0, st, g->off, g->okey, g->dag_off, g->dag_adj,
                                   list_b, cnt_b, kMidMaxD, L.ctl + 2, res, res3, none);
        }
        GPM_LAUNCH_CHECK("k_lg4<512>");
        {
            Span sp("k_lg4<256>", st);
            const dim3 grid((unsigned)cu_count() * 8);
            if (em)
                hipLaunchKernelGGL((k_lg4<kMidMaxD, kMidThreads, true, false>), grid,
                                   dim3(kMidThreads), 0, st, g->off, g->okey, g->dag_off, g->dag_adj,
                                   list_m, cnt_m, 0, L.ctl + 1, res, res3, *em);
            else
                hipLaunchKernelGGL((k_lg4<kMidMaxD, kMidThreads, false, false>), grid,
                                   dim3(kMidThreads), 0, st, g->off, g->okey, g->dag_off, g->dag_adj,
                                   list_m, cnt_m, 0, L.ctl + 1, res, res3, none);
        }
        GPM_LAUNCH_CHECK("k_lg4<256>");
        return GPM_OK;
    }
    gpm_status rc = lg5_class<kBigMaxD, kBigThreads>(g, k, L, list_b, cnt_b, L.rowoff_b, L.rows_b,
                                                     L.units + 0, L.toff_b, L.ctl + 2, res, res3,
                                                     res4, em, st, "k_lg_build<1024>",
                                                     k == 5 ? "k_lg5<1024>" : "k_lgk<1024>");
    if (rc) return rc;
    {
        Span sp(k == 5 ? "k_lg5_mid<256>" : "k_lgk_mid<256>", st);
        const dim3 grid((unsigned)cu_count() * 8);
        if (em)
            hipLaunchKernelGGL((k_lg5_mid<kMidMaxD, kMidThreads, true>), grid, dim3(kMidThreads), 0,
                               st, g->off, g->okey, g->dag_off, g->dag_adj, list_m, cnt_m, k - 5,
                               L.ctl + 6, res, res3, res4, *em);
        else
            hipLaunchKernelGGL((k_lg5_mid<kMidMaxD, kMidThreads, false>), grid, dim3(kMidThreads),
                               0, st, g->off, g->okey, g->dag_off, g->dag_adj, list_m, cnt_m, k - 5,
                               L.ctl + 6, res, res3, res4, RowEmitter{});
    }
    GPM_LAUNCH_CHECK("k_lg5_mid");
    return GPM_OK;
}

}  // namespace gpm
