// Batched 3- and 4-motif counting of many small graphs in one launch.
//
// The G graphs are one union graph g whose graph i owns vertices
// voff[i] .. voff[i+1]-1.  A persistent grid of teams (one workgroup per
// graph at a time, graphs popped from an atomic cursor) computes every step
// of the motif path for its graph entirely on chip: the graph's adjacency
// becomes bit rows in LDS (row v = neighbours of v, ceil(n/64) words), and
//   degrees             d_v = |A_v|
//   per-edge triangles  T_uv = |A_u & A_v|               (Section 5)
//   local-count sums    the four per-edge sums of the motif path
//   4-cliques           sum over triangles u < v < w of |A_u & A_v & A_w & above(w)|
//   4-cycles            sum over x, z < x of C(|A_x & A_z & below(x)|, 2)
//                       (each cycle once, from its largest vertex x and the
//                       opposite vertex z; the middles lie below x)
// are combined into the induced counts with the same exact identities as the
// single-graph path, and written to the graph's row of the output.
#include "gpm_internal.h"

#include <algorithm>

namespace gpm {

namespace {

typedef unsigned __int128 u128;

constexpr int kSmallN = 256;    // one wave per graph
constexpr int kSmallNT = 64;
constexpr int kLargeN = GPM_BATCH_MAX_VERTICES;   // one 256-thread workgroup per graph
constexpr int kLargeNT = 256;

enum BatchFlags : unsigned long long {
    B_DIVISION = 1,       // an exact division of the combining identities failed
    B_TOO_LARGE = 64,     // graph has more than GPM_BATCH_MAX_VERTICES vertices
    B_BAD_RANGE = 128,    // voff not ascending or beyond n
    B_CROSS_EDGE = 256,   // an edge leaves the graph's vertex range
};

__device__ __forceinline__ uint64_t below_mask(int32_t x, int32_t w) {
    // bits < x within word w
    const int32_t lo = w * 64;
    if (x <= lo) return 0ull;
    if (x >= lo + 64) return ~0ull;
    return (1ull << (x - lo)) - 1ull;
}

template <int NMAX, int NT>
struct BatchLds {
    static constexpr int W = NMAX / 64;
    uint64_t rows[NMAX * W];
    int32_t deg[NMAX];
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

template <int NMAX, int NT, bool STATIC>
__global__ void __launch_bounds__(NT) k_batch(const int32_t *__restrict__ off,
                                              const int32_t *__restrict__ adj,
                                              const int32_t *__restrict__ voff, int32_t G,
                                              int32_t n, int32_t k, int32_t nmin,
                                              uint32_t *cursor, unsigned long long *counts) {
    constexpr int W = NMAX / 64;
    __shared__ BatchLds<NMAX, NT> sh;
    const int tid = threadIdx.x;
    const int width = k == 3 ? 3 : 7;
    uint32_t gi = STATIC ? blockIdx.x : 0;
    for (;;) {
        if (!STATIC) {
            if (tid == 0) sh.task = atomicAdd(cursor, 1u);
            __syncthreads();
            gi = sh.task;
            __syncthreads();
        }
        if ((int32_t)gi >= G) break;
        const int32_t v0 = voff[gi], v1 = voff[gi + 1];
        unsigned long long *out = counts + (int64_t)gi * width;
        const bool bad_range = v0 < 0 || v1 < v0 || v1 > n;
        const int32_t ng = bad_range ? 0 : v1 - v0;
        const bool mine = !bad_range && ng > nmin && ng <= NMAX;
        if (!mine) {
            // the atomic-cursor kernel (every graph passes through it) reports
            // graphs that no kernel can take
            if (!bad_range && ng > kLargeN && tid == 0 && !STATIC) {
                for (int q = 0; q < width; q++) out[q] = 0;
                out[width - 1] = B_TOO_LARGE;
            }
            if (bad_range && tid == 0 && !STATIC) {
                for (int q = 0; q < width; q++) out[q] = 0;
                out[width - 1] = B_BAD_RANGE;
            }
            gi += STATIC ? gridDim.x : 0;
            continue;
        }
        const int32_t Wg = (ng + 63) >> 6;
        for (int32_t i = tid; i < ng * W; i += NT) sh.rows[i] = 0ull;
        if (tid == 0) sh.flags = 0;
        __syncthreads();
        const int32_t a0 = off[v0], a1 = off[v1];
        for (int32_t e = a0 + tid; e < a1; e += NT) {
            // row owner of arc e: binary search over the graph's offsets
            int32_t lo = v0, hi = v1;
            while (hi - lo > 1) {
                const int32_t mid = (lo + hi) >> 1;
                if (off[mid] <= e) lo = mid; else hi = mid;
            }
            const int32_t w = adj[e];
            if (w < v0 || w >= v1) {
                atomicOr(&sh.flags, (unsigned long long)B_CROSS_EDGE);
                continue;
            }
            const int32_t u = lo - v0, x = w - v0;
            atomicOr((unsigned long long *)&sh.rows[u * W + (x >> 6)], 1ull << (x & 63));
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
        // edges u < v, one per thread
        for (int32_t e = a0 + tid; e < a1; e += NT) {
            int32_t lo = v0, hi = v1;
            while (hi - lo > 1) {
                const int32_t mid = (lo + hi) >> 1;
                if (off[mid] <= e) lo = mid; else hi = mid;
            }
            const int32_t w = adj[e];
            if (w < v0 || w >= v1) continue;
            const int32_t u = lo - v0, v = w - v0;
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
                        for (int32_t r = x >> 6; r < Wg; r++)
                            k4 += __popcll(ru[r] & rv[r] & rx[r] & ~below_mask(x + 1, r));
                    }
                }
            }
        }
        if (k == 4) {
            // 4-cycles from their largest vertex x and opposite vertex z < x
            const int64_t npairs = (int64_t)ng * (ng - 1) / 2;
            for (int64_t p = tid; p < npairs; p += NT) {
                int64_t x = (int64_t)((1.0 + sqrt(1.0 + 8.0 * (double)p)) * 0.5);
                while (x * (x - 1) / 2 > p) x--;
                while ((x + 1) * x / 2 <= p) x++;
                const int32_t z = (int32_t)(p - x * (x - 1) / 2);
                const uint64_t *rx = sh.rows + x * W, *rz = sh.rows + z * W;
                uint64_t c = 0;
                for (int32_t q = 0; q < Wg; q++)
                    c += __popcll(rx[q] & rz[q] & below_mask((int32_t)x, q));
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
        gi += STATIC ? gridDim.x : 0;
    }
}

}  // namespace

gpm_status batch_workspace_bytes(int32_t G, int32_t k, uint64_t *bytes) {
    (void)G;
    (void)k;
    *bytes = 256;   // one cursor word
    return GPM_OK;
}

gpm_status batch_run(const gpm_graph *g, const int32_t *d_voff, int32_t G, int32_t k, void *ws,
                     uint64_t ws_bytes, unsigned long long *d_counts, hipStream_t st) {
    if (ws_bytes < 256) return fail(GPM_OUT_OF_MEMORY, "workspace smaller than required");
    uint32_t *cursor = static_cast<uint32_t *>(ws);
    GPM_HIP(fill_u32(cursor, 0, 1, st));
    {
        Span sp("k_batch<256>", st);
        hipLaunchKernelGGL((k_batch<kSmallN, kSmallNT, false>),
                           dim3((unsigned)std::min<int64_t>(G, (int64_t)cu_count() * 16)),
                           dim3(kSmallNT), 0, st, g->off, g->adj, d_voff, G, g->n, k, -1, cursor,
                           d_counts);
    }
    GPM_LAUNCH_CHECK("k_batch<256>");
    {
        Span sp("k_batch<1024>", st);
        hipLaunchKernelGGL((k_batch<kLargeN, kLargeNT, true>),
                           dim3((unsigned)std::min<int64_t>(G, (int64_t)cu_count())),
                           dim3(kLargeNT), 0, st, g->off, g->adj, d_voff, G, g->n, k, kSmallN,
                           cursor, d_counts);
    }
    GPM_LAUNCH_CHECK("k_batch<1024>");
    return GPM_OK;
}

}  // namespace gpm
