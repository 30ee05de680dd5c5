// Induced 5-motif counts by formulas (the counting-by-formula approach the
// paper names in Section 7; the method here follows the idea of ESCAPE,
// Pinar, Seshadhri and Vishal, WWW 2017: non-induced counts, most of them
// from local counts, then exact back-substitution).
//
// For the 21 connected 5-vertex graphs H (classes in gpm_motif_class_pattern
// order: by edge count, then by canonical code), N(P) = number of subgraphs
// (edge sets) isomorphic to P and I(H) = number of induced copies satisfy
//     N(P) = sum over H of c(P, H) I(H),
// c(P, H) = number of spanning subgraphs of H isomorphic to P (c(H, H) = 1,
// zero unless H has more edges), so I follows by back-substitution from the
// densest class down.  The matrix c is built on the host by brute force over
// the edge subsets of each class.
//
// Fifteen N(P) have closed forms in local counts: degrees d, per-edge
// triangle counts T_e (the Section 5 local counts, from the triangle
// kernels), per vertex t_v = triangles at v, s_v = sum of the neighbours'
// degrees and q_v = sum of (neighbour degree - 1)^2, the totals T, K4 and
// N(C4), D = sum over edges of C(T_e, 2) (diamonds), two sums over the
// 4-cycles C (of the degrees of their vertices, of the triangle counts of
// their edges), two over the triangles and two over the 4-cliques:
//   star K1,4   sum_v C(d_v, 4)
//   chair       sum over ordered arcs (c, x) of C(d_c - 1, 2)(d_x - 1) - T_cx (d_c - 2)
//   5-path      sum_c [(s_c - d_c)^2 - q_c] / 2 - (2 sum_v t_v d_v - 9T) - 4 N(C4)
//   cricket     sum_c t_c C(d_c - 2, 2)
//   bull        sum_e T_e [(d_x - 2)(d_y - 2) - (T_e - 1)]
//   banner      sum_C sum_{v in C} (d_v - 2) - 2D          (4-cycle with a pendant)
//   tadpole     sum_c t_c (s_c - d_c) - (2 sum_v t_v d_v - 6T) - 2 sum_e T_e (T_e - 1)
//   dart        sum_e C(T_e, 2)(d_x + d_y - 6)
//   kite        sum over triangles of sum over their edges e of (T_e - 1) d(opposite vertex)
//               - 4D - 12 K4                                  (pendant at a diamond's tip)
//   bowtie      sum_v C(t_v, 2) - 2 sum_e C(T_e, 2)
//   house       sum_C sum_{e in C} T_e - 4D
//   K4+pendant  sum over 4-cliques of sum over their vertices of (d_v - 3)
//   book        sum_e C(T_e, 3)                               (three triangles on an edge)
//   gem         sum over triangles of sum over their vertices v of (T_vp - 1)(T_vq - 1)
//               - 12 K4                                       (a vertex joined to a 4-path)
//   K4+ear      sum over 4-cliques of sum over their edges of (T_e - 2)
//                                                (a vertex joined to two vertices of a K4)
// (each derived by counting the choices of the pattern's free vertices
// around a cut vertex, a cut edge, a 4-cycle or a triangle, and subtracting
// the choices that collide: a chord of a 4-cycle, a fourth vertex closing a
// K4).  A sixteenth, the 5-cycle, comes from closed walks (Harary and
// Manvel, 1971): a closed 5-walk is a 5-cycle (ten walks each) or a
// triangle with one edge walked back and forth at one of its vertices, so
//   5-cycle     [tr(A^5) - 30 T - 10 sum_v (d_v - 2) t_v] / 10
// with tr(A^5) from each vertex's row of A^2, and a seventeenth from the
// same rows: a K_{2,3} is its two degree-3 vertices and three of their
// common neighbours,
//   K_{2,3}     sum over vertex pairs u < v of C(c(u, v), 3)
// with c(u, v) = (A^2)_uv, and an eighteenth: class 16, two non-adjacent
// vertices c, d joined to a, b, e with a ~ b, is its pair {c, d} with an
// edge among their common neighbours and one more of them,
//   class 16    sum over pairs {c, d} of E_cd (c(c, d) - 2)
//               = [sum over triangles {c, a, b}, d != c in N(a) & N(b)
//                  of c(c, d)] / 2 - 2D
// (E_cd the edges among the pair's common neighbours), and a nineteenth:
// K5 minus an edge is a triangle t (its degree-4 vertices) with two
// vertices adjacent to all of it,
//   K5 - e      sum over triangles t of C(k4(t), 2)
// (k4(t) the vertices adjacent to all of t), and a twentieth: the wheel
// is its hub (its one vertex of degree 4) and a 4-cycle among the hub's
// neighbours,
//   wheel       sum over vertices i of N(C4) in G[N(i)]
// (graphs of up to kTrace5MaxN vertices; above, these five are counted
// directly as induced patterns by the general plan).  K5 is counted by the
// clique kernels.
#include "gpm_internal.h"

#include <algorithm>
#include <mutex>
#include <vector>

namespace gpm {

gpm_status clique_workspace_bytes(const gpm_graph *g, int32_t k, bool list, uint64_t *bytes);
gpm_status clique_run(const gpm_graph *g, int32_t k, bool list, void *ws, uint64_t ws_bytes,
                      unsigned long long *d_count, int32_t *d_buf, uint64_t cap,
                      unsigned long long *d_result, hipStream_t st);
gpm_status triangle_arc_counts(const gpm_graph *g, void *ws, uint64_t ws_bytes, uint32_t *te,
                               unsigned long long *tri, hipStream_t st);
gpm_status c4_workspace_bytes(const gpm_graph *g, bool list, uint64_t *bytes);
gpm_status c4_run(const gpm_graph *g, bool list, void *ws, uint64_t ws_bytes,
                  unsigned long long *out128, int32_t *d_buf, uint64_t cap,
                  unsigned long long *d_result, hipStream_t st,
                  const uint32_t *tsym = nullptr, unsigned long long *cs = nullptr);
uint64_t generic_workspace_bytes(const gpm_graph *g);
gpm_status generic_count(const gpm_graph *g, const gpm_pattern *p, void *ws, uint64_t ws_bytes,
                         unsigned long long *out, hipStream_t st);
gpm_status motif_class_pattern(int k, int idx, gpm_pattern *out);

namespace {

typedef unsigned __int128 u128;

constexpr int kClasses = 21;
constexpr int kBlock = 256;

// Classes with a closed form, and the accumulator pair (plus, minus) of each.
enum Formula : int { F_STAR, F_CHAIR, F_PATH, F_CRICKET, F_BULL, F_BANNER, F_TADPOLE, F_DART,
                     F_KITE, F_BOWTIE, F_HOUSE, F_K4PEND, F_BOOK, F_GEM, F_K4TWO, F_C5, F_K23,
                     F_TWIN, F_K5E, F_WHEEL, F_COUNT };
constexpr int kFormulaClass[F_COUNT] = {0, 1, 2, 3, 4, 5, 6, 8, 9, 11, 12, 13, 14, 15, 17, 7, 10,
                                        16, 19, 18};
// the formulas of the 5-cycle, K_{2,3}, class 16, K5 minus an edge and the
// wheel need dense per-vertex arrays in LDS (a row of A^2, neighbour
// bitmaps, 16-bit counters): graphs of up to kTrace5MaxN vertices (above,
// the five are counted directly)
constexpr int32_t kTrace5MaxN = 65536;
constexpr int kK5Class = 20;

struct Back {
    uint16_t c[kClasses][kClasses];   // c[P][H], spanning copies of P in H
    int32_t formula_of[kClasses];     // F_* or -1 (counted directly)
};

// Accumulators: 2 u64 words per u128.
enum Acc : int {
    A_PLUS = 0,                       // F_COUNT u128: positive parts
    A_MINUS = A_PLUS + 2 * F_COUNT,   // F_COUNT u128: subtracted parts
    A_TRI = A_MINUS + 2 * F_COUNT,    // u64: triangles (from the arc counts)
    A_C4 = A_TRI + 2,                 // u128: 4-cycles (edge sets)
    A_CYC = A_C4 + 2,                 // 2 u128: 4-cycle sums (degrees, doubled; edge triangles)
    A_K4 = A_CYC + 4,                 // u64: 4-cliques
    A_DIR = A_K4 + 2,                 // kClasses u64: induced counts of the direct classes
    A_CURSOR = A_DIR + kClasses,      // u64: the wheel kernel's work cursor
    A_TCURSOR = A_CURSOR + 1,         // u64: the A^2-row kernel's task cursor
    A_WORDS = A_TCURSOR + 1,
};

__device__ __forceinline__ u128 binom2(uint64_t n) { return n < 2 ? 0 : (u128)n * (n - 1) / 2; }

// Orders a wave's LDS writes before its later reads.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
__device__ __forceinline__ u128 binom4(uint64_t n) {
    return n < 4 ? 0 : (u128)n * (n - 1) / 2 * (n - 2) / 3 * (n - 3) / 4;
}

// Per vertex: t_v from the arc triangle counts (each arc adds its count to
// both ends; every triangle at v lies on two of v's arcs).
__global__ void k_vertex_tri(const int32_t *__restrict__ dag_src, const int32_t *__restrict__ dag_adj,
                             const uint32_t *__restrict__ te, int64_t m,
                             unsigned long long *__restrict__ t2) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t c = te[e];
        if (c) {
            atomicAdd(&t2[dag_src[e]], (unsigned long long)c);
            atomicAdd(&t2[dag_adj[e]], (unsigned long long)c);
        }
    }
}

// One wave per vertex: s_v, q_v over the neighbours, then the vertex terms
// of the formulas.
__global__ void __launch_bounds__(kBlock) k_f5_vertex(const int32_t *__restrict__ off,
                                                      const int32_t *__restrict__ adj, int32_t n,
                                                      const unsigned long long *__restrict__ t2,
                                                      unsigned long long *acc) {
    const int lane = lane_id();
    const int64_t wave0 = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * (kBlock / kWave);
    u128 plus[F_COUNT] = {}, minus[F_COUNT] = {};
    for (int64_t v = wave0; v < n; v += nwaves) {
        const int32_t s0 = off[v], dv = off[v + 1] - s0;
        uint64_t s = 0, q = 0;
        for (int32_t i = lane; i < dv; i += kWave) {
            const int32_t w = adj[s0 + i];
            const uint64_t dw = (uint64_t)(off[w + 1] - off[w]);
            s += dw;
            q += (dw - 1) * (dw - 1);
        }
        s = wave_sum(s);
        q = wave_sum(q);
        if (lane != 0) continue;
        const uint64_t d = (uint64_t)dv, t = t2[v] / 2;
        plus[F_STAR] += binom4(d);
        // 5-path: pairs of neighbours b < b' of the middle, (d_b - 1)(d_b' - 1)
        const u128 sd = (u128)(s - d);
        plus[F_PATH] += (sd * sd - (u128)q) / 2;
        minus[F_PATH] += (u128)2 * t * d;
        if (d >= 2) plus[F_CRICKET] += (u128)t * binom2(d - 2);
        plus[F_TADPOLE] += (u128)t * (s - d);
        minus[F_TADPOLE] += (u128)2 * t * d;
        plus[F_BOWTIE] += binom2(t);
        // 5-cycles: 10 sum_v (d_v - 2) t_v, with t2 = 2 t_v
        if (d >= 2) minus[F_C5] += (u128)5 * (d - 2) * t2[v];
    }
#pragma unroll
    for (int f = 0; f < F_COUNT; f++) {
        const u128 p = wave_sum_u128(plus[f]), mm = wave_sum_u128(minus[f]);
        if (lane == 0) {
            if (p) atomic_add_u128(acc + A_PLUS + 2 * f, p);
            if (mm) atomic_add_u128(acc + A_MINUS + 2 * f, mm);
        }
    }
}

// tr(A^5) = sum over vertices i of the closed 5-walks at i,
//   (A^5)_ii = sum over j of P2(i, j) sum over k in N(j) of P2(i, k)
// with P2(i, .) = row i of A^2 (2-walk counts; A^2 is symmetric), and
// N(K_{2,3}) = sum over vertex pairs i < j of C(P2(i, j), 3) (a K_{2,3} is
// its two degree-3 vertices and three of their common neighbours), and for
// class 16 (two non-adjacent vertices c, d joined to a, b, e with a ~ b)
//   S = sum over triangles {c, a, b} and common neighbours d != c of a, b
//       of P2(c, d),
// twice the sum over pairs {c, d} of (edges inside their common
// neighbourhood) x (its size): each triangle at c, with c as the row; and
// for K5 minus an edge, a triangle t with two vertices adjacent to all of
// it, C(k4(t), 2) summed over the triangles, k4(t) = the common neighbours
// of a and b also adjacent to c (each triangle is met at each of its three
// vertices, so the sum is three times the count).  A
// workgroup per task (i, part) builds P2(i, .) densely in LDS (n 16-bit
// counters, no list of the j it reaches: a ballot over the counter words
// finds them); part 0 sums over the reached j and their neighbours; each part marks N(i) in an LDS bitmap and walks the
// triangles at i whose end a of larger degree is among its kTracePart
// neighbours of i (each wave with the bitmap of its a, two triangles at a
// time, 32 lanes on each), then clears what it set.  The tasks come from a
// cursor, so a hub's parts run side by side.  P2 <= n, so each product
// fits 64 bits; the sums are 128-bit.
constexpr int32_t kTracePart = 128;             // neighbours a per triangle-walk task
constexpr int kTriLanes = 32;                   // lanes per triangle walked
constexpr int kTriGroups = kWave / kTriLanes;   // triangles per wave at a time

template <int NT, bool SHARED>
__global__ void __launch_bounds__(NT) k_f5_trace5(const int32_t *__restrict__ off,
                                                  const int32_t *__restrict__ adj, int32_t n,
                                                  int32_t nparts, unsigned long long *acc) {
    extern __shared__ uint4 s_trace[];
    // P2(i, j) < n <= 65536: 16-bit counters packed two to a word (hw4
    // words, a multiple of 4), then the bitmaps; the reached j are the
    // nonzero counters, found by scanning the words
    const int32_t hw = (n + 1) / 2, hw4 = (hw + 3) / 4 * 4;
    uint32_t *p2w = reinterpret_cast<uint32_t *>(s_trace);
    uint32_t *nbm = p2w + hw4;                           // bitmap of N(i)
    const int32_t nbw = (n + 31) / 32;
    auto p2 = [&](int32_t j) -> uint32_t { return (p2w[j >> 1] >> ((j & 1) * 16)) & 0xFFFFu; };
    __shared__ int64_t s_task;
    const int tid = threadIdx.x, lane = lane_id(), wid = tid / kWave;
    const int grp = lane / kTriLanes, gl = lane % kTriLanes;
    constexpr int NW = NT / kWave;
    // this wave's bitmap of N(a) (SHARED: one for the workgroup, after N(i))
    uint32_t *wbm = nbm + (int64_t)(1 + (SHARED ? 0 : wid)) * nbw;
    for (int32_t i = tid; i < hw4; i += NT) p2w[i] = 0;
    for (int32_t i = tid; i < (SHARED ? 2 : 1 + NW) * nbw; i += NT) nbm[i] = 0;
    __syncthreads();
    u128 tr = 0, k23 = 0, twin = 0, k5e = 0;
    // tasks (i, part) from a cursor, the parts from the last down, so that
    // the vertices of highest degree start first
    const int64_t ntasks = (int64_t)n * nparts;
    for (;;) {
        if (tid == 0) s_task = (int64_t)atomicAdd(acc + A_TCURSOR, 1ull);
        __syncthreads();
        const int64_t t = s_task;
        __syncthreads();
        if (t >= ntasks) break;
        const int32_t part = nparts - 1 - (int32_t)(t / n), i = (int32_t)(t % n);
        const int32_t si = off[i], di = off[i + 1] - si;
        const int32_t a_lo = part * kTracePart;
        if (part > 0 && a_lo >= di) continue;
        const int32_t a_hi = a_lo + kTracePart < di ? a_lo + kTracePart : di;
        // 2-walks i - x - j: a wave per middle x, lanes over N(x)
        for (int32_t a = wid; a < di; a += NW) {
            const int32_t x = adj[si + a], sx = off[x], dx = off[x + 1] - sx;
            for (int32_t b = lane; b < dx; b += kWave) {
                const int32_t j = adj[sx + b];
                atomicAdd(&p2w[j >> 1], 1u << ((uint32_t)(j & 1) * 16u));
            }
        }
        __syncthreads();
        if (part == 0) {
            for (int32_t w = tid; w < hw; w += NT) {
                const uint32_t v = p2w[w];
                if (!v) continue;
#pragma unroll
                for (int h = 0; h < 2; h++) {
                    const int32_t j = 2 * w + h;
                    const uint64_t c = (v >> (16 * h)) & 0xFFFFu;
                    if (j > i && c >= 3) k23 += (u128)(c * (c - 1) * (c - 2) / 6);
                }
            }
            // sum over the reached j of P2(i, j) times the P2 of j's
            // neighbours, (A^3)_ij; the term is symmetric in i and j, so each
            // pair j != i is taken once, doubled, at its end of larger
            // (degree, id), walking the row of the other; a wave per 64
            // counter words, their nonzero ones by ballot
            for (int32_t w0 = wid * kWave; w0 < hw; w0 += NW * kWave) {
                const uint32_t v = w0 + lane < hw ? p2w[w0 + lane] : 0u;
                uint64_t mask = __ballot(v != 0u);
                while (mask) {
                    const int src = __builtin_ctzll(mask);
                    mask &= mask - 1ull;
                    const uint32_t vv = __shfl(v, src, kWave);
#pragma unroll
                    for (int h = 0; h < 2; h++) {
                        const uint64_t pv = (vv >> (16 * h)) & 0xFFFFu;
                        const int32_t j = 2 * (w0 + src) + h;
                        if (!pv) continue;
                        const int32_t sj = off[j], dj = off[j + 1] - sj;
                        if (j != i && (dj > di || (dj == di && j > i))) continue;
                        const uint64_t pj = pv << (j != i);
                        uint64_t sum = 0;
                        for (int32_t b = lane; b < dj; b += kWave) sum += p2(adj[sj + b]);
                        tr += (u128)(pj * sum);
                    }
                }
            }
        }
        for (int32_t a = tid; a < di; a += NT) {
            const int32_t x = adj[si + a];
            atomicOr(&nbm[x >> 5], 1u << (x & 31));
        }
        __syncthreads();
        // triangles {i, a, b}: a wave per a, with N(a) marked in its own
        // bitmap; each triangle taken at its end of larger (degree, id), a,
        // walking the other end's row and testing N(a) (and N(i)) in LDS:
        // the common neighbours d != i of a and b add P2(i, d)
        // the triangles of a whose lower ends are N(a)'s entries b0 .. b0+63
        auto walk = [&](int32_t a, int32_t sa, int32_t da, int32_t b0, const uint32_t *abm) {
            const int32_t b = b0 + lane < da ? adj[sa + b0 + lane] : -1;
            bool tri = false;
            if (b >= 0 && ((nbm[b >> 5] >> (b & 31)) & 1u)) {
                const int32_t db = off[b + 1] - off[b];
                tri = db < da || (db == da && b < a);
            }
            // kTriGroups triangles at a time, kTriLanes lanes each
            uint64_t mask = __ballot(tri);
            while (mask) {
                uint64_t mm = mask;
                for (int g = 0; g < grp && mm; g++) mm &= mm - 1ull;
                const bool live = mm != 0ull;
                const int src = live ? __builtin_ctzll(mm) : 0;
                for (int g = 0; g < kTriGroups && mask; g++) mask &= mask - 1ull;
                const int32_t bb = __shfl(b, src, kWave);
                const int32_t sb = live ? off[bb] : 0, db = live ? off[bb + 1] - sb : 0;
                uint32_t q = 0;   // common neighbours of a, b adjacent to i
                for (int32_t k = gl; k < db; k += kTriLanes) {
                    const int32_t d = adj[sb + k];
                    if (d != i && ((abm[d >> 5] >> (d & 31)) & 1u)) {
                        twin += (u128)p2(d);
                        q += (nbm[d >> 5] >> (d & 31)) & 1u;
                    }
                }
#pragma unroll
                for (int o = kTriLanes / 2; o > 0; o >>= 1) q += __shfl_xor(q, o, kWave);
                if (gl == 0) k5e += (u128)q * (q - (q > 0)) / 2;
            }
        };
        if constexpr (!SHARED) {
            // a wave per a, N(a) in the wave's own bitmap
            for (int32_t ai = a_lo + wid; ai < a_hi; ai += NW) {
                const int32_t a = adj[si + ai], sa = off[a], da = off[a + 1] - sa;
                for (int32_t k = lane; k < da; k += kWave) {
                    const int32_t x = adj[sa + k];
                    atomicOr(&wbm[x >> 5], 1u << (x & 31));
                }
                wave_sync();
                for (int32_t b0 = 0; b0 < da; b0 += kWave) walk(a, sa, da, b0, wbm);
                wave_sync();
                for (int32_t k = lane; k < da; k += kWave) wbm[adj[sa + k] >> 5] = 0u;
                wave_sync();
            }
        } else {
            // the workgroup on one a at a time, N(a) in one shared bitmap,
            // the waves on its entries 64 at a time
            uint32_t *abm = nbm + nbw;
            for (int32_t ai = a_lo; ai < a_hi; ai++) {
                const int32_t a = adj[si + ai], sa = off[a], da = off[a + 1] - sa;
                for (int32_t k = tid; k < da; k += NT) {
                    const int32_t x = adj[sa + k];
                    atomicOr(&abm[x >> 5], 1u << (x & 31));
                }
                __syncthreads();
                for (int32_t b0 = wid * kWave; b0 < da; b0 += NT) walk(a, sa, da, b0, abm);
                __syncthreads();
                for (int32_t k = tid; k < da; k += NT) abm[adj[sa + k] >> 5] = 0u;
                __syncthreads();
            }
        }
        __syncthreads();
        uint4 *p2w4 = reinterpret_cast<uint4 *>(p2w);
        for (int32_t k = tid; k < hw4 / 4; k += NT) p2w4[k] = make_uint4(0u, 0u, 0u, 0u);
        for (int32_t a = tid; a < di; a += NT) nbm[adj[si + a] >> 5] = 0u;
        __syncthreads();
    }
    tr = wave_sum_u128(tr);
    k23 = wave_sum_u128(k23);
    twin = wave_sum_u128(twin);
    k5e = wave_sum_u128(k5e);
    if (lane == 0 && tr) atomic_add_u128(acc + A_PLUS + 2 * F_C5, tr);
    if (lane == 0 && k23) atomic_add_u128(acc + A_PLUS + 2 * F_K23, k23);
    if (lane == 0 && twin) atomic_add_u128(acc + A_PLUS + 2 * F_TWIN, twin);
    if (lane == 0 && k5e) atomic_add_u128(acc + A_PLUS + 2 * F_K5E, k5e);
}

// The wheel (a hub joined to all four vertices of a 4-cycle) has one
// vertex of degree 4, its hub, so its copies are the pairs (i, 4-cycle in
// G[N(i)]).  A 4-cycle x-p-y-q is taken at its largest vertex x, y the
// vertex opposite x: C(c(x, y), 2) over the y < x in N(i), c(x, y) = the
// common neighbours p < x of x and y in N(i).  A wave per arc (i, x), the
// arcs taken kWheelArcs at a time from a cursor (consecutive arcs share i,
// whose neighbours stay marked in the wave's LDS bitmap, with the number of
// marks before each bitmap word); c(x, y) in 16-bit counters packed two to
// an LDS word and indexed by y's position in N(i) (c < d(i) < 65536), so a
// wave's counters take 2 bytes per vertex of the largest degree, not per
// vertex of the graph; each increment adds the count before it (0 + 1 + ...
// + (c - 1) = C(c, 2)), then the first d(i) counters are cleared.  Rows are
// sorted, so only their entries below x are read, kWheelU chunks of 64 in
// flight per wave.
constexpr int kWheelArcs = 4;
constexpr int kWheelU = 4;

// LDS words per wave: counters (max degree), bitmap (n bits), 16-bit
// prefix per bitmap word; each part a multiple of 4 words
__host__ __device__ constexpr int32_t wheel_count_words(int32_t maxdeg) {
    return ((maxdeg + 1) / 2 + 3) / 4 * 4;
}
__host__ __device__ constexpr int32_t wheel_bitmap_words(int32_t n) {
    return ((n + 31) / 32 + 3) / 4 * 4;
}
__host__ __device__ constexpr int32_t wheel_words_per_wave(int32_t n, int32_t maxdeg) {
    return wheel_count_words(maxdeg) + wheel_bitmap_words(n) + (wheel_bitmap_words(n) / 2 + 3) / 4 * 4;
}

__device__ __forceinline__ bool marked(const uint32_t *bm, int32_t v) {
    return (bm[v >> 5] >> (v & 31)) & 1u;
}

__global__ void __launch_bounds__(kBlock) k_f5_wheel(const int32_t *__restrict__ off,
                                                     const int32_t *__restrict__ adj, int32_t n,
                                                     int32_t maxdeg, int64_t arcs,
                                                     unsigned long long *acc) {
    extern __shared__ uint4 s_wheel[];
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    const int32_t cw = wheel_count_words(maxdeg), ww = wheel_words_per_wave(n, maxdeg);
    const int32_t nbw = (n + 31) / 32;
    uint32_t *cnt = reinterpret_cast<uint32_t *>(s_wheel) + (int64_t)wid * ww;
    uint4 *cnt4 = reinterpret_cast<uint4 *>(cnt);
    uint32_t *bm = cnt + cw;                    // N(i)
    uint16_t *pf = reinterpret_cast<uint16_t *>(bm + wheel_bitmap_words(n));   // marks before
    for (int32_t k = lane; k < ww; k += kWave) cnt[k] = 0u;
    wave_sync();
    u128 sum = 0;
    int32_t cur = -1;   // the vertex whose neighbours are marked
    const int64_t nblocks = (arcs + kWheelArcs - 1) / kWheelArcs;
    for (;;) {
        unsigned long long r = 0;
        if (lane == 0) r = atomicAdd(acc + A_CURSOR, 1ull);
        const int64_t b = __shfl((int64_t)r, 0, kWave);
        if (b >= nblocks) break;
        const int64_t t0 = b * kWheelArcs, t1 = t0 + kWheelArcs < arcs ? t0 + kWheelArcs : arcs;
        // the row holding arc t0: off[i] <= t0 < off[i + 1]
        int32_t lo = 0, hi = n;
        while (hi - lo > 1) {
            const int32_t mid = (lo + hi) >> 1;
            if (off[mid] <= t0) lo = mid; else hi = mid;
        }
        int32_t i = lo;
        for (int64_t t = t0; t < t1; t++) {
            while (off[i + 1] <= t) i++;
            if (i != cur) {
                if (cur >= 0)
                    for (int32_t k = off[cur] + lane; k < off[cur + 1]; k += kWave)
                        bm[adj[k] >> 5] = 0u;
                wave_sync();
                for (int32_t k = off[i] + lane; k < off[i + 1]; k += kWave) {
                    const int32_t v = adj[k];
                    atomicOr(&bm[v >> 5], 1u << (v & 31));
                }
                wave_sync();
                int32_t carry = 0;
                for (int32_t w0 = 0; w0 < nbw; w0 += kWave) {
                    const int32_t c = w0 + lane < nbw ? __popc(bm[w0 + lane]) : 0;
                    const int32_t incl = wave_incl_scan(c);
                    if (w0 + lane < nbw) pf[w0 + lane] = (uint16_t)(carry + incl - c);
                    carry += __shfl(incl, kWave - 1, kWave);
                }
                wave_sync();
                cur = i;
            }
            const int32_t x = adj[t], sx = off[x], dx = off[x + 1] - sx;
            bool touched = false;
            for (int32_t k0 = 0; k0 < dx; k0 += kWave) {
                const int32_t p = k0 + lane < dx ? adj[sx + k0 + lane] : INT32_MAX;
                uint64_t mask = __ballot(p < x && marked(bm, p));
                touched |= mask != 0ull;
                while (mask) {
                    const int src = __builtin_ctzll(mask);
                    mask &= mask - 1ull;
                    const int32_t pp = __shfl(p, src, kWave);
                    const int32_t sp = off[pp], dp = off[pp + 1] - sp;
                    for (int32_t j0 = 0; j0 < dp; j0 += kWave * kWheelU) {
                        int32_t y[kWheelU];
#pragma unroll
                        for (int u = 0; u < kWheelU; u++) {
                            const int32_t j = j0 + u * kWave + lane;
                            y[u] = j < dp ? adj[sp + j] : INT32_MAX;
                        }
#pragma unroll
                        for (int u = 0; u < kWheelU; u++) {
                            if (y[u] < x) {
                                const uint32_t wv = bm[y[u] >> 5], b = (uint32_t)(y[u] & 31);
                                if ((wv >> b) & 1u) {
                                    // y's position in N(i)
                                    const int32_t r = pf[y[u] >> 5] + __popc(wv & ((1u << b) - 1u));
                                    const uint32_t sh = (uint32_t)(r & 1) * 16u;
                                    const uint32_t old = atomicAdd(&cnt[r >> 1], 1u << sh);
                                    sum += (old >> sh) & 0xFFFFu;
                                }
                            }
                        }
                        if (__ballot(y[kWheelU - 1] >= x)) break;   // the rest are >= x
                    }
                }
                if (__ballot(p >= x)) break;
            }
            if (touched) {   // the first d(i) counters: ceil(d(i) / 8) uint4
                const int32_t nclr = (off[i + 1] - off[i] + 7) / 8;
                wave_sync();
                for (int32_t k = lane; k < nclr; k += kWave) cnt4[k] = make_uint4(0u, 0u, 0u, 0u);
                wave_sync();
            }
        }
    }
    sum = wave_sum_u128(sum);
    if (lane == 0 && sum) atomic_add_u128(acc + A_PLUS + 2 * F_WHEEL, sum);
}

// One thread per undirected edge (an arc of the DAG): the edge terms.
__global__ void __launch_bounds__(kBlock) k_f5_edge(const int32_t *__restrict__ off,
                                                    const int32_t *__restrict__ dag_src,
                                                    const int32_t *__restrict__ dag_adj,
                                                    const uint32_t *__restrict__ te, int64_t m,
                                                    unsigned long long *acc) {
    const int lane = lane_id();
    u128 plus[F_COUNT] = {}, minus[F_COUNT] = {};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e0 = (int64_t)blockIdx.x * blockDim.x; e0 < m; e0 += stride) {
        const int64_t e = e0 + threadIdx.x;
        if (e >= m) continue;
        const int32_t x = dag_src[e], y = dag_adj[e];
        const uint64_t dx = (uint64_t)(off[x + 1] - off[x]), dy = (uint64_t)(off[y + 1] - off[y]);
        const uint64_t T = te[e];
        // chair, both orientations: centre c, its neighbour x on the long arm
        plus[F_CHAIR] += binom2(dx - 1) * (dy - 1) + binom2(dy - 1) * (dx - 1);
        if (T) {
            // a triangle on the edge puts both ends at degree >= 2
            minus[F_CHAIR] += (u128)T * ((dx - 2) + (dy - 2));
            plus[F_BULL] += (u128)T * ((dx - 2) * (dy - 2));
            minus[F_BULL] += (u128)T * (T - 1);
            minus[F_TADPOLE] += (u128)2 * T * (T - 1);
            const u128 diamonds = binom2(T);
            minus[F_BOWTIE] += 2 * diamonds;
            minus[F_BANNER] += 2 * diamonds;
            minus[F_HOUSE] += 4 * diamonds;
            minus[F_KITE] += 4 * diamonds;
            minus[F_TWIN] += 4 * diamonds;
            // two triangles on the edge put both ends at degree >= 3
            if (T >= 2) plus[F_DART] += diamonds * (dx + dy - 6);
            if (T >= 3) plus[F_BOOK] += diamonds * (T - 2) / 3;
        }
    }
#pragma unroll
    for (int f = 0; f < F_COUNT; f++) {
        const u128 p = wave_sum_u128(plus[f]), mm = wave_sum_u128(minus[f]);
        if (lane == 0) {
            if (p) atomic_add_u128(acc + A_PLUS + 2 * f, p);
            if (mm) atomic_add_u128(acc + A_MINUS + 2 * f, mm);
        }
    }
}

// tsym[a] = triangles on the edge of arc a of the symmetric CSR, from the
// counts per arc of the DAG (one thread per DAG arc, a binary search in
// each end's row).
__global__ void __launch_bounds__(kBlock) k_tsym(const int32_t *__restrict__ off,
                                                 const int32_t *__restrict__ adj,
                                                 const int32_t *__restrict__ dag_src,
                                                 const int32_t *__restrict__ dag_adj,
                                                 const uint32_t *__restrict__ te, int64_t m,
                                                 uint32_t *__restrict__ tsym) {
    auto find = [&](int32_t u, int32_t v) {
        int32_t lo = off[u], hi = off[u + 1];
        while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            if (adj[mid] < v) lo = mid + 1; else hi = mid;
        }
        return lo;
    };
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t u = dag_src[e], v = dag_adj[e];
        const uint32_t c = te[e];
        tsym[find(u, v)] = c;
        tsym[find(v, u)] = c;
    }
}

// The triangle terms of the kite and the gem.  One wave per DAG arc
// u -> v: lanes take w in N+(v) and look it up in N+(u) (rows ascending),
// so each triangle u -> v -> w, u -> w is met once, with its three arcs.
__global__ void __launch_bounds__(kBlock) k_f5_tri(const int32_t *__restrict__ off,
                                                   const int32_t *__restrict__ dag_off,
                                                   const int32_t *__restrict__ dag_src,
                                                   const int32_t *__restrict__ dag_adj,
                                                   const uint32_t *__restrict__ te, int64_t m,
                                                   unsigned long long *acc) {
    const int lane = lane_id();
    const int64_t wave0 = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * (kBlock / kWave);
    uint64_t kite = 0, gem = 0;
    for (int64_t e = wave0; e < m; e += nwaves) {
        const int32_t u = dag_src[e], v = dag_adj[e];
        const uint32_t t_uv = te[e];
        if (t_uv == 0) continue;   // wave-uniform
        const int32_t su = dag_off[u], du = dag_off[u + 1] - su;
        const int32_t sv = dag_off[v], dv = dag_off[v + 1] - sv;
        const uint64_t deg_u = (uint64_t)(off[u + 1] - off[u]);
        const uint64_t deg_v = (uint64_t)(off[v + 1] - off[v]);
        for (int32_t i = lane; i < dv; i += kWave) {
            const int32_t w = dag_adj[sv + i];
            int32_t lo = 0, hi = du;
            while (lo < hi) {
                const int32_t mid = (lo + hi) >> 1;
                if (dag_adj[su + mid] < w) lo = mid + 1; else hi = mid;
            }
            if (lo < du && dag_adj[su + lo] == w) {
                const uint64_t a = t_uv - 1u, b = te[su + lo] - 1u, c = te[sv + i] - 1u;
                const uint64_t deg_w = (uint64_t)(off[w + 1] - off[w]);
                // edges uv, uw, vw; opposite vertices w, v, u
                kite += a * deg_w + b * deg_v + c * deg_u;
                // centres u (edges uv, uw), v (uv, vw), w (uw, vw)
                gem += a * b + a * c + b * c;
            }
        }
    }
    const u128 k = wave_sum_u128((u128)kite), g = wave_sum_u128((u128)gem);
    if (lane == 0) {
        if (k) atomic_add_u128(acc + A_PLUS + 2 * F_KITE, k);
        if (g) atomic_add_u128(acc + A_PLUS + 2 * F_GEM, g);
    }
}

// The 4-clique terms.  One wave per DAG arc u -> v: lanes find the w of
// N+(v) in N+(u) (the triangles u, v, w); for each such w in turn, lanes
// take x in N+(w) and look it up in N+(u) and N+(v).  Each 4-clique
// u -> v -> w -> x is met once, with its six arcs.
__global__ void __launch_bounds__(kBlock) k_f5_k4(const int32_t *__restrict__ off,
                                                  const int32_t *__restrict__ dag_off,
                                                  const int32_t *__restrict__ dag_src,
                                                  const int32_t *__restrict__ dag_adj,
                                                  const uint32_t *__restrict__ te, int64_t m,
                                                  unsigned long long *acc) {
    const int lane = lane_id();
    const int64_t wave0 = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * (kBlock / kWave);
    auto find = [&](int32_t s0, int32_t len, int32_t x) {   // index in the row, or -1
        int32_t lo = 0, hi = len;
        while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            if (dag_adj[s0 + mid] < x) lo = mid + 1; else hi = mid;
        }
        return lo < len && dag_adj[s0 + lo] == x ? lo : -1;
    };
    uint64_t pend = 0, two = 0;
    for (int64_t e = wave0; e < m; e += nwaves) {
        const int32_t u = dag_src[e], v = dag_adj[e];
        if (te[e] < 2) continue;   // wave-uniform: an edge of a 4-clique has two triangles
        const int32_t su = dag_off[u], du = dag_off[u + 1] - su;
        const int32_t sv = dag_off[v], dv = dag_off[v + 1] - sv;
        const uint64_t deg_uv = (uint64_t)(off[u + 1] - off[u]) + (uint64_t)(off[v + 1] - off[v]);
        for (int32_t i0 = 0; i0 < dv; i0 += kWave) {
            const int32_t i = i0 + lane;
            int32_t iw = -1, w = -1;
            if (i < dv) {
                w = dag_adj[sv + i];
                iw = find(su, du, w);
            }
            uint64_t mask = __ballot(iw >= 0);
            while (mask) {
                const int src = __builtin_ctzll(mask);
                mask &= mask - 1;
                const int32_t ww = __shfl(w, src, 64), iu_w = __shfl(iw, src, 64);
                const int32_t iv_w = i0 + src;
                const int32_t sw = dag_off[ww], dw = dag_off[ww + 1] - sw;
                const uint64_t t3 = (uint64_t)te[e] + te[su + iu_w] + te[sv + iv_w];
                const uint64_t deg_w = (uint64_t)(off[ww + 1] - off[ww]);
                for (int32_t j = lane; j < dw; j += kWave) {
                    const int32_t x = dag_adj[sw + j];
                    const int32_t ixu = find(su, du, x);
                    if (ixu < 0) continue;
                    const int32_t ixv = find(sv, dv, x);
                    if (ixv < 0) continue;
                    const uint64_t deg_x = (uint64_t)(off[x + 1] - off[x]);
                    pend += deg_uv + deg_w + deg_x - 12u;
                    two += t3 + te[su + ixu] + te[sv + ixv] + te[sw + j] - 12u;
                }
            }
        }
    }
    const u128 a = wave_sum_u128((u128)pend), b = wave_sum_u128((u128)two);
    if (lane == 0) {
        if (a) atomic_add_u128(acc + A_PLUS + 2 * F_K4PEND, a);
        if (b) atomic_add_u128(acc + A_PLUS + 2 * F_K4TWO, b);
    }
}

__device__ __forceinline__ u128 load128(const unsigned long long *p) {
    return ((u128)p[1] << 64) | p[0];
}

// Totals of the formulas, then back-substitution from the densest class.
// out[0..20] = induced counts, out[21] = status (1: a formula or a
// subtraction went negative, 2: a count does not fit 64 bits).
__global__ void k_f5_combine(const unsigned long long *acc, Back B, unsigned long long *out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    unsigned long long bad = 0;
    const u128 T = (u128)acc[A_TRI];
    const u128 nc4 = load128(acc + A_C4);
    const u128 cyc_deg2 = load128(acc + A_CYC), cyc_tri = load128(acc + A_CYC + 2);
    const u128 k4 = (u128)acc[A_K4];
    if (cyc_deg2 & 1) bad |= 1;   // twice a sum
    u128 N[kClasses];
    for (int h = 0; h < kClasses; h++) {
        const int f = B.formula_of[h];
        if (f < 0) {
            N[h] = 0;
            continue;
        }
        u128 p = load128(acc + A_PLUS + 2 * f), mm = load128(acc + A_MINUS + 2 * f);
        // the global terms
        if (f == F_PATH) {
            p += 9 * T;
            mm += 4 * nc4;
        }
        if (f == F_TADPOLE) p += 6 * T;
        if (f == F_BANNER) {
            p += cyc_deg2 / 2;
            mm += 8 * nc4;
        }
        if (f == F_HOUSE) p += cyc_tri;
        if (f == F_KITE || f == F_GEM) mm += 12 * k4;
        if (f == F_C5) mm += 30 * T;   // 5 tr(A^3) = 30 T
        if (p < mm) bad |= 1;
        N[h] = p - mm;
        if (f == F_C5) {   // ten closed 5-walks per 5-cycle
            if (N[h] % 10) bad |= 1;
            N[h] /= 10;
        }
        if (f == F_TWIN) {   // both orders of each pair {c, d}
            if (N[h] & 1) bad |= 1;
            N[h] /= 2;
        }
        if (f == F_K5E) {   // each triangle at each of its vertices
            if (N[h] % 3) bad |= 1;
            N[h] /= 3;
        }
    }
    // densest first: a direct class is its count, a formula class its N
    // minus the copies inside denser induced subgraphs
    u128 I[kClasses];
    for (int h = kClasses - 1; h >= 0; h--) {
        if (B.formula_of[h] < 0) {
            I[h] = (u128)acc[A_DIR + h];
        } else {
            u128 sub = 0;
            for (int k = h + 1; k < kClasses; k++) sub += (u128)B.c[h][k] * I[k];
            if (N[h] < sub) bad |= 1;
            I[h] = N[h] - sub;
        }
        if (I[h] >> 64) bad |= 2;
        out[h] = (unsigned long long)I[h];
    }
    out[kClasses] = bad;
}

__global__ void k_copy_u64(const unsigned long long *src, unsigned long long *dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = *src;
}

// Host: canonical form of a 5-vertex edge set (smallest sorted edge list
// over the 120 vertex orders).
uint32_t canon5(const int (*e)[2], int ne) {
    int p[5] = {0, 1, 2, 3, 4};
    uint32_t best = ~0u;
    do {
        uint32_t code = 0;
        for (int i = 0; i < ne; i++) {
            int a = p[e[i][0]], b = p[e[i][1]];
            if (a > b) std::swap(a, b);
            // bit of pair (a, b), a < b, in a 10-bit set
            const int bit = a * (9 - a) / 2 + (b - a - 1);
            code |= 1u << bit;
        }
        best = std::min(best, code);
    } while (std::next_permutation(p, p + 5));
    return best;
}

bool connected5(const int (*e)[2], int ne) {
    int reach = 1;
    for (int it = 0; it < 5; it++)
        for (int i = 0; i < ne; i++) {
            const int a = 1 << e[i][0], b = 1 << e[i][1];
            if ((reach & a) || (reach & b)) reach |= a | b;
        }
    return reach == 31;
}

const Back &back_matrix() {
    static Back B;
    static bool made = false;
    static std::mutex mu;
    std::lock_guard<std::mutex> lock(mu);
    if (made) return B;
    gpm_pattern cls[kClasses];
    uint32_t code[kClasses];
    for (int h = 0; h < kClasses; h++) {
        motif_class_pattern(5, h, &cls[h]);
        int e[10][2];
        for (int i = 0; i < cls[h].n_edges; i++) {
            e[i][0] = cls[h].edges[i][0];
            e[i][1] = cls[h].edges[i][1];
        }
        code[h] = canon5(e, cls[h].n_edges);
    }
    for (int p = 0; p < kClasses; p++)
        for (int h = 0; h < kClasses; h++) B.c[p][h] = 0;
    for (int h = 0; h < kClasses; h++) {
        const int ne = cls[h].n_edges;
        for (uint32_t sub = 1; sub < (1u << ne); sub++) {
            int e[10][2], k = 0, seen = 0;
            for (int i = 0; i < ne; i++)
                if ((sub >> i) & 1u) {
                    e[k][0] = cls[h].edges[i][0];
                    e[k][1] = cls[h].edges[i][1];
                    seen |= (1 << e[k][0]) | (1 << e[k][1]);
                    k++;
                }
            if (seen != 31 || !connected5(e, k)) continue;
            const uint32_t c = canon5(e, k);
            for (int p = 0; p < kClasses; p++)
                if (code[p] == c) B.c[p][h]++;
        }
    }
    for (int h = 0; h < kClasses; h++) B.formula_of[h] = -1;
    for (int f = 0; f < F_COUNT; f++) B.formula_of[kFormulaClass[f]] = f;
    made = true;
    return B;
}

struct F5Ws {
    unsigned long long *acc, *t2;
    uint32_t *te, *tsym;
    void *shared;
    uint64_t shared_bytes, bytes;
};

F5Ws f5_layout(const gpm_graph *g, void *base) {
    F5Ws W{};
    Carve c(base, ~0ull);
    W.acc = c.take<unsigned long long>(A_WORDS);
    W.t2 = c.take<unsigned long long>((uint64_t)g->n + 1);
    W.te = c.take<uint32_t>((uint64_t)g->m + 1);
    W.tsym = c.take<uint32_t>(2 * (uint64_t)g->m + 1);
    uint64_t b3 = 0, b5 = 0, bc4 = 0;
    uint64_t b4 = 0;
    clique_workspace_bytes(g, 3, false, &b3);
    clique_workspace_bytes(g, 4, false, &b4);
    clique_workspace_bytes(g, 5, false, &b5);
    c4_workspace_bytes(g, false, &bc4);
    W.shared_bytes = std::max({b3, b4, b5, bc4, generic_workspace_bytes(g)});
    W.shared = c.take<char>(W.shared_bytes);
    W.bytes = c.used;
    return W;
}

unsigned grid_for(int64_t items, int per_block, int cap_per_cu) {
    int64_t b = (items + per_block - 1) / per_block;
    int64_t cap = (int64_t)cu_count() * cap_per_cu;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

}  // namespace

gpm_status motif_formula_workspace_bytes(const gpm_graph *g, int32_t k, uint64_t *bytes) {
    if (k != 5) return fail(GPM_UNSUPPORTED, "formula motif counting is for k = 5");
    *bytes = f5_layout(g, nullptr).bytes;
    return GPM_OK;
}

gpm_status motif_formula_count(const gpm_graph *g, int32_t k, void *ws, uint64_t ws_bytes,
                               unsigned long long *d_counts, hipStream_t st) {
    if (k != 5) return fail(GPM_UNSUPPORTED, "formula motif counting is for k = 5");
    F5Ws W = f5_layout(g, ws);
    if (W.bytes > ws_bytes) return fail(GPM_OUT_OF_MEMORY, "workspace smaller than required");
    // the 5-cycle, K_{2,3}, class 16 and K5 minus an edge from the rows of
    // A^2 where they fit in LDS, else counted directly
    Back B = back_matrix();
    const int32_t n = g->n;
    const int64_t m = g->m;
    const bool trace5 = n <= kTrace5MaxN;
    if (!trace5) {
        B.formula_of[kFormulaClass[F_C5]] = -1;
        B.formula_of[kFormulaClass[F_K23]] = -1;
        B.formula_of[kFormulaClass[F_TWIN]] = -1;
        B.formula_of[kFormulaClass[F_K5E]] = -1;
        B.formula_of[kFormulaClass[F_WHEEL]] = -1;
    }
    GPM_HIP(fill_u32(W.acc, 0, 2 * (uint64_t)A_WORDS, st));
    GPM_HIP(fill_u32(W.t2, 0, 2 * ((uint64_t)n + 1), st));
    if (m > 0) GPM_HIP(fill_u32(W.te, 0, (uint64_t)m, st));
    // local counts: triangles per edge (and their total), per vertex
    gpm_status rc = triangle_arc_counts(g, W.shared, W.shared_bytes, W.te, W.acc + A_TRI, st);
    if (rc) return rc;
    {
        Span sp("k_f5_local", st);
        if (m > 0) {
            hipLaunchKernelGGL(k_vertex_tri, dim3(grid_for(m, kBlock, 8)), dim3(kBlock), 0, st,
                               g->dag_src, g->dag_adj, W.te, m, W.t2);
            hipLaunchKernelGGL(k_f5_edge, dim3(grid_for(m, kBlock, 8)), dim3(kBlock), 0, st,
                               g->off, g->dag_src, g->dag_adj, W.te, m, W.acc);
            hipLaunchKernelGGL(k_tsym, dim3(grid_for(m, kBlock, 8)), dim3(kBlock), 0, st, g->off,
                               g->adj, g->dag_src, g->dag_adj, W.te, m, W.tsym);
            hipLaunchKernelGGL(k_f5_tri, dim3(grid_for(m, kBlock / kWave, 16)), dim3(kBlock), 0,
                               st, g->off, g->dag_off, g->dag_src, g->dag_adj, W.te, m, W.acc);
            hipLaunchKernelGGL(k_f5_k4, dim3(grid_for(m, kBlock / kWave, 16)), dim3(kBlock), 0,
                               st, g->off, g->dag_off, g->dag_src, g->dag_adj, W.te, m, W.acc);
        }
        hipLaunchKernelGGL(k_f5_vertex, dim3(grid_for(n, kBlock / kWave, 8)), dim3(kBlock), 0,
                           st, g->off, g->adj, n, W.t2, W.acc);
    }
    GPM_LAUNCH_CHECK("k_f5_local");
    if (trace5 && m > 0) {
        Span sp("k_f5_trace5", st);
        // 16-bit P2 counters, the bitmaps of N(i) and of each wave's N(a)
        // in 16-wave workgroups; where those bitmaps do not fit (above
        // about 39,700 vertices), one N(a) bitmap that the workgroup's waves
        // share, a at a time
        const size_t p2_bytes = (size_t)(((n + 1) / 2 + 3) / 4 * 4) * 4;
        const size_t bm_bytes = (size_t)((n + 31) / 32) * 4;
        const bool shared = p2_bytes + bm_bytes * (1 + 1024 / kWave) > 160 * 1024;
        const size_t shmem = p2_bytes + bm_bytes * (shared ? 2 : 1 + 1024 / kWave);
        const int per_cu =
            (int)std::max<int64_t>(1, std::min<int64_t>(8, (160 * 1024) / (int64_t)(shmem + 1024)));
        // a vertex's triangles split into parts of kTracePart neighbours
        // a, each part a task that builds the row of A^2 again
        const int32_t nparts = std::max<int32_t>(1, (g->max_degree + kTracePart - 1) / kTracePart);
        const dim3 grid(grid_for((int64_t)n * nparts, 1, per_cu));
        if (shared)
            hipLaunchKernelGGL((k_f5_trace5<1024, true>), grid, dim3(1024), shmem, st, g->off,
                               g->adj, n, nparts, W.acc);
        else
            hipLaunchKernelGGL((k_f5_trace5<1024, false>), grid, dim3(1024), shmem, st, g->off,
                               g->adj, n, nparts, W.acc);
    }
    GPM_LAUNCH_CHECK("k_f5_trace5");
    if (trace5 && m > 0) {
        Span sp("k_f5_wheel", st);
        // per wave: the counters c(x, .) and the bitmap of N(i); up to 4
        // waves per workgroup, as many as their LDS allows
        const size_t per_wave = (size_t)wheel_words_per_wave(n, g->max_degree) * 4;
        const int waves = (int)std::max<size_t>(1, std::min<size_t>(4, (160 * 1024) / per_wave));
        const size_t shmem = per_wave * waves;
        const int per_cu =
            (int)std::max<int64_t>(1, std::min<int64_t>(8, (160 * 1024) / (int64_t)(shmem + 1024)));
        const int64_t arcs = 2 * m;
        hipLaunchKernelGGL(k_f5_wheel,
                           dim3(grid_for((arcs + kWheelArcs - 1) / kWheelArcs, waves, per_cu)),
                           dim3(waves * kWave), shmem, st, g->off, g->adj, n, g->max_degree,
                           arcs, W.acc);
    }
    GPM_LAUNCH_CHECK("k_f5_wheel");
    // 4-cycles (edge sets) and the sums over them
    rc = c4_run(g, false, W.shared, W.shared_bytes, W.acc + A_C4, nullptr, 0, nullptr, st,
                W.tsym, W.acc + A_CYC);
    if (rc) return rc;
    rc = clique_run(g, 4, false, W.shared, W.shared_bytes, W.acc + A_K4, nullptr, 0, nullptr, st);
    if (rc) return rc;
    // the direct classes: K5 by the clique kernels, the rest by the general
    // plan as vertex-induced patterns
    for (int h = 0; h < kClasses; h++) {
        if (B.formula_of[h] >= 0) continue;
        unsigned long long *slot = W.acc + A_DIR + h;
        if (h == kK5Class) {
            rc = clique_run(g, 5, false, W.shared, W.shared_bytes, slot, nullptr, 0, nullptr, st);
        } else {
            gpm_pattern p;
            motif_class_pattern(5, h, &p);
            p.flags = GPM_VERTEX_INDUCED;
            rc = generic_count(g, &p, W.shared, W.shared_bytes, slot, st);
        }
        if (rc) return rc;
    }
    hipLaunchKernelGGL(k_f5_combine, dim3(1), dim3(64), 0, st, W.acc, B, d_counts);
    GPM_LAUNCH_CHECK("k_f5_combine");
    return GPM_OK;
}

}  // namespace gpm
