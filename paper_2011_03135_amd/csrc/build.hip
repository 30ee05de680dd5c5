// Canonical CSR build and degree-ordered orientation, entirely on the device.
//
// Input: a raw undirected edge stream (u[i], v[i]).  Output (graph storage):
//   off/adj        symmetric, loop-free, duplicate-free, rows ascending
//                  (the input form assumed in Section 6, input-graph table);
//   dag_off/adj    arcs u -> v with (deg u, u) < (deg v, v), rows ascending
//                  (degree-based orientation, Appendix B.2);
//   dag_src        the source vertex of every arc.
//
// Pipeline (one stream, no host round trip until the final size read-back):
//   arcs into buckets of consecutive source ids (LDS histograms per tile)
//   -> per bucket: row offsets and arcs into rows (LDS counters)
//   -> per-row sort + unique (wave bitonic in registers for <= 64 entries,
//      wave bitonic in LDS for <= 2048, workgroup bitmap for longer rows)
//   -> scan unique counts -> compact rows -> count out-arcs -> scan -> fill.
#include "gpm_internal.h"

#include <algorithm>
#include <climits>
#include <new>

namespace gpm {

namespace {

enum Flag : int {
    F_ERR = 0,        // nonzero: an input id was out of range
    F_BIG_COUNT = 1,  // rows routed to the bitmap sorter
    F_MAX_DEG = 2,
    F_MAX_OUT = 3,
    F_MED_COUNT = 4,  // rows routed to the one-row-per-wave register sort
    F_DEG16 = 5,      // vertices of degree above 65535
    F_WORDS = 16,
};

constexpr int kBlock = 256;                 // 4 waves
constexpr int kWavesPerBlock = kBlock / kWave;

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ void __launch_bounds__(kBlock) k_count_raw(const int32_t *__restrict__ u,
                                                      const int32_t *__restrict__ v, int64_t E,
                                                      int32_t n, int32_t *cnt, uint32_t *flags) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * kBlock;
    for (; i < E; i += stride) {
        int32_t a = u[i], b = v[i];
        if ((uint32_t)a >= (uint32_t)n || (uint32_t)b >= (uint32_t)n) {
            atomicOr(&flags[F_ERR], 1u);
            continue;
        }
        if (a == b) continue;
        atomicAdd(&cnt[a], 1);
        atomicAdd(&cnt[b], 1);
    }
}

__global__ void __launch_bounds__(kBlock) k_scatter_raw(const int32_t *__restrict__ u,
                                                        const int32_t *__restrict__ v, int64_t E,
                                                        int32_t n, const int32_t *raw_off,
                                                        int32_t *cursor, int32_t *raw_adj) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * kBlock;
    for (; i < E; i += stride) {
        int32_t a = u[i], b = v[i];
        if ((uint32_t)a >= (uint32_t)n || (uint32_t)b >= (uint32_t)n || a == b) continue;
        int32_t pa = atomicAdd(&cursor[a], 1);
        raw_adj[raw_off[a] + pa] = b;
        int32_t pb = atomicAdd(&cursor[b], 1);
        raw_adj[raw_off[b] + pb] = a;
    }
}

// ------------------------------------------- bucketed arc distribution --
// Arcs (both directions of every raw edge, loops dropped) go to rows in
// three passes without global atomics on hot vertices: arcs are first
// counted and moved into buckets of 2^S consecutive source ids (one LDS
// histogram per tile of edges, one global atomic per tile and bucket), then
// each bucket's block counts its sources in LDS, writes the row offsets and
// places the arcs inside the bucket's own range of the row array.
constexpr int kTileEdges = 8192;     // raw edges per tile
constexpr int kMaxBuckets = 4096;    // LDS histogram of a tile
constexpr int kMaxBucketIds = 16384; // LDS counters of a bucket (2^S <= this)
constexpr int kBucketNT = 1024;

__global__ void __launch_bounds__(kBlock) k_bucket_count(const int32_t *__restrict__ u,
                                                         const int32_t *__restrict__ v,
                                                         int64_t E, int32_t n, int32_t S,
                                                         int32_t nb, int32_t *bucket_cnt,
                                                         uint32_t *flags) {
    __shared__ int32_t hist[kMaxBuckets];
    const int64_t ntiles = (E + kTileEdges - 1) / kTileEdges;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        for (int b = threadIdx.x; b < nb; b += kBlock) hist[b] = 0;
        __syncthreads();
        const int64_t e1 = min(E, (t + 1) * (int64_t)kTileEdges);
        for (int64_t i = t * (int64_t)kTileEdges + threadIdx.x; i < e1; i += kBlock) {
            const int32_t a = u[i], b = v[i];
            if ((uint32_t)a >= (uint32_t)n || (uint32_t)b >= (uint32_t)n) {
                atomicOr(&flags[F_ERR], 1u);
                continue;
            }
            if (a == b) continue;
            atomicAdd(&hist[a >> S], 1);
            atomicAdd(&hist[b >> S], 1);
        }
        __syncthreads();
        for (int b = threadIdx.x; b < nb; b += kBlock)
            if (hist[b]) atomicAdd(&bucket_cnt[b], hist[b]);
        __syncthreads();
    }
}

// Moves a tile's arcs into their buckets through LDS: the arcs are first
// placed in bucket order in LDS (LDS histogram, block prefix, one global
// atomic per bucket for the tile's share), then copied out with consecutive
// threads writing consecutive slots of a bucket, so each bucket's share
// leaves as one contiguous run instead of scattered 4-byte stores.  LDS
// (dynamic): hist, prefix and global base per bucket, then the tile's arcs.
constexpr int kScatterNT = 1024;

__global__ void __launch_bounds__(kScatterNT) k_bucket_scatter(const int32_t *__restrict__ u,
                                                               const int32_t *__restrict__ v,
                                                               int64_t E, int32_t n, int32_t S,
                                                               int32_t nb, int32_t tile_edges,
                                                               int32_t *bucket_cur, int32_t *bsrc,
                                                               int32_t *bdst) {
    constexpr int PER = kMaxBuckets / kScatterNT;
    extern __shared__ int32_t sm[];
    int32_t *hist = sm, *lpre = hist + nb, *gbase = lpre + nb + 1;
    int32_t *s_sum = gbase + nb, *ssrc = s_sum + kScatterNT / kWave;
    int32_t *sdst = ssrc + 2 * tile_edges;
    const int tid = threadIdx.x;
    const int64_t ntiles = (E + tile_edges - 1) / tile_edges;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        for (int b = tid; b < nb; b += kScatterNT) hist[b] = 0;
        __syncthreads();
        const int64_t e0 = t * (int64_t)tile_edges, e1 = min(E, e0 + tile_edges);
        for (int64_t i = e0 + tid; i < e1; i += kScatterNT) {
            const int32_t a = u[i], b = v[i];
            if ((uint32_t)a >= (uint32_t)n || (uint32_t)b >= (uint32_t)n || a == b) continue;
            atomicAdd(&hist[a >> S], 1);
            atomicAdd(&hist[b >> S], 1);
        }
        __syncthreads();
        int32_t val[PER];
#pragma unroll
        for (int q = 0; q < PER; q++) {
            const int b = tid * PER + q;
            val[q] = b < nb ? hist[b] : 0;
        }
        block_prefix<kScatterNT, PER>(val, nb, lpre, s_sum);
        // the tile's share of each bucket; hist becomes the LDS cursor
        for (int b = tid; b < nb; b += kScatterNT) {
            const int32_t c = hist[b];
            gbase[b] = c ? atomicAdd(&bucket_cur[b], c) : 0;
            hist[b] = lpre[b];
        }
        __syncthreads();
        for (int64_t i = e0 + tid; i < e1; i += kScatterNT) {
            const int32_t a = u[i], b = v[i];
            if ((uint32_t)a >= (uint32_t)n || (uint32_t)b >= (uint32_t)n || a == b) continue;
            const int32_t pa = atomicAdd(&hist[a >> S], 1);
            ssrc[pa] = a;
            sdst[pa] = b;
            const int32_t pb = atomicAdd(&hist[b >> S], 1);
            ssrc[pb] = b;
            sdst[pb] = a;
        }
        __syncthreads();
        const int32_t total = lpre[nb];
        for (int32_t i = tid; i < total; i += kScatterNT) {
            int32_t lo = 0, hi = nb;   // last bucket with lpre <= i
            while (hi - lo > 1) {
                const int32_t mid = (lo + hi) >> 1;
                if (lpre[mid] <= i) lo = mid; else hi = mid;
            }
            const int32_t g = gbase[lo] + (i - lpre[lo]);
            bsrc[g] = ssrc[i];
            bdst[g] = sdst[i];
        }
        __syncthreads();
    }
}

// Dynamic LDS of k_bucket_scatter for nb buckets and a tile of te edges.
size_t scatter_lds_bytes(int32_t nb, int32_t te) {
    return ((size_t)3 * nb + 1 + kScatterNT / kWave + 4 * (size_t)te) * 4;
}

// One block per bucket: row offsets of its 2^S sources and their arcs.
__global__ void __launch_bounds__(kBucketNT) k_bucket_rows(const int32_t *__restrict__ bucket_off,
                                                           const int32_t *__restrict__ bsrc,
                                                           const int32_t *__restrict__ bdst,
                                                           int32_t n, int32_t S, int32_t nb,
                                                           int32_t *raw_off, int32_t *raw_adj) {
    constexpr int PER = kMaxBucketIds / kBucketNT;
    __shared__ int32_t cnt[kMaxBucketIds + 1];
    __shared__ int32_t s_sum[kBucketNT / kWave];
    const int32_t ids = 1 << S;
    for (int32_t b = blockIdx.x; b < nb; b += gridDim.x) {
        const int32_t base = b << S;
        const int32_t a0 = bucket_off[b], a1 = bucket_off[b + 1];
        for (int32_t i = threadIdx.x; i < ids; i += kBucketNT) cnt[i] = 0;
        __syncthreads();
        for (int32_t i = a0 + threadIdx.x; i < a1; i += kBucketNT) atomicAdd(&cnt[bsrc[i] - base], 1);
        __syncthreads();
        int32_t val[PER];
#pragma unroll
        for (int q = 0; q < PER; q++) {
            const int32_t i = threadIdx.x * PER + q;
            val[q] = i < ids ? cnt[i] : 0;
        }
        __syncthreads();
        // exclusive prefix of the counts: cnt[i] becomes the first slot of row base+i
        block_prefix<kBucketNT, PER>(val, ids, cnt, s_sum);
        for (int32_t i = threadIdx.x; i < ids; i += kBucketNT) {
            const int32_t vtx = base + i;
            if (vtx < n) raw_off[vtx] = a0 + cnt[i];
        }
        __syncthreads();
        for (int32_t i = a0 + threadIdx.x; i < a1; i += kBucketNT) {
            const int32_t p = atomicAdd(&cnt[bsrc[i] - base], 1);
            raw_adj[a0 + p] = bdst[i];
        }
        __syncthreads();
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) raw_off[n] = bucket_off[nb];
}

// Sorts row entries held one per lane of each group of G lanes (lanes past
// the row hold INT_MAX) ascending.
template <int G>
__device__ __forceinline__ int32_t group_bitonic_sort(int32_t x) {
    const int lane = lane_id() & (G - 1);
#pragma unroll
    for (int k = 2; k <= G; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            int32_t y = __shfl_xor(x, j, 64);
            bool ascending = (lane & k) == 0;
            bool lower = (lane & j) == 0;
            int32_t lo = x < y ? x : y, hi = x < y ? y : x;
            x = (lower == ascending) ? lo : hi;
        }
    }
    return x;
}

constexpr int kSmallRow = 16;   // rows sorted by a 16-lane group, 4 per wave
constexpr int kScanRow = 512;   // rows up to this length sort in registers within a row scan
constexpr int kRegRow = 2048;   // rows up to this length sort in registers, a wave each

// Sorts + uniques one row of L <= 64 R entries in place with one wave, all in
// registers: entry i sits in lane i % 64 of x[i / 64], so bitonic partners
// closer than 64 are a lane exchange and farther ones a register pair of
// the same lane.  The row is read in full before any write, so in place is
// safe.  Returns the unique count.
template <int R>
__device__ int32_t wave_sort_row_regs(int32_t *r, int32_t L) {
    const int lane = lane_id();
    int32_t x[R];
#pragma unroll
    for (int q = 0; q < R; q++) x[q] = q * kWave + lane < L ? r[q * kWave + lane] : INT_MAX;
#pragma unroll
    for (int k = 2; k <= R * kWave; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j >= kWave) {
                const int jr = j / kWave;
#pragma unroll
                for (int q = 0; q < R; q++) {
                    if (q & jr) continue;
                    const bool ascending = ((q * kWave) & k) == 0;   // k >= 128 here
                    const int32_t a = x[q], b = x[q | jr];
                    const int32_t lo = a < b ? a : b, hi = a < b ? b : a;
                    x[q] = ascending ? lo : hi;
                    x[q | jr] = ascending ? hi : lo;
                }
            } else {
                const bool lower = (lane & j) == 0;
#pragma unroll
                for (int q = 0; q < R; q++) {
                    const int32_t y = __shfl_xor(x[q], j, 64);
                    const bool ascending = ((q * kWave + lane) & k) == 0;
                    const int32_t lo = x[q] < y ? x[q] : y, hi = x[q] < y ? y : x[q];
                    x[q] = (lower == ascending) ? lo : hi;
                }
            }
        }
    }
    int32_t count = 0;
    int32_t last = INT_MAX;   // the previous register's lane-63 entry
#pragma unroll
    for (int q = 0; q < R; q++) {
        const int32_t i = q * kWave + lane;
        int32_t prev = __shfl_up(x[q], 1, 64);
        if (lane == 0) prev = last;
        const bool keep = i < L && (i == 0 || x[q] != prev);
        const uint64_t mask = __ballot(keep);
        if (keep) r[count + lanes_below(mask)] = x[q];
        count += __popcll(mask);
        last = __builtin_amdgcn_readlane(x[q], 63);
    }
    return count;
}

// Short rows: each 16-lane group sorts + uniques one row of at most 16
// entries in place (4 consecutive rows per wave).  Rows beyond kScanRow go
// to lists (up to kRegRow the list of the wave-per-row register sort, the
// bitmap sorter's beyond); the rest are left to k_sort_rows' row scan.  Most
// rows of power-law graphs are short.
__global__ void __launch_bounds__(kBlock) k_sort_small_rows(const int32_t *__restrict__ raw_off,
                                                            int32_t *raw_adj, int32_t n,
                                                            int32_t *ucnt, int32_t *med_list,
                                                            int32_t *big_list, uint32_t *flags) {
    const int lane = lane_id(), gl = lane & (kSmallRow - 1), grp = lane / kSmallRow;
    const int64_t wave0 = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
    constexpr int kRows = kWave / kSmallRow;
    for (int64_t r0 = wave0 * kRows; r0 < n; r0 += nwaves * kRows) {
        const int64_t row = r0 + grp;
        const bool live = row < n;
        const int32_t s = live ? raw_off[row] : 0;
        const int32_t L = live ? raw_off[row + 1] - s : 0;
        const bool small = L <= kSmallRow;
        int32_t *r = raw_adj + s;
        int32_t x = small && gl < L ? r[gl] : INT_MAX;
        x = group_bitonic_sort<kSmallRow>(x);
        const int32_t prev = __shfl(x, lane - 1, 64);
        const bool keep = small && gl < L && (gl == 0 || x != prev);
        const uint64_t mask = __ballot(keep);
        const uint32_t gmask = (uint32_t)(mask >> (grp * kSmallRow)) & ((1u << kSmallRow) - 1u);
        if (keep) r[__popc(gmask & ((1u << gl) - 1u))] = x;
        if (live && gl == 0) {
            if (small) ucnt[row] = __popc(gmask);
            else if (L > kRegRow) big_list[atomicAdd(&flags[F_BIG_COUNT], 1u)] = (int32_t)row;
            else if (L > kScanRow) med_list[atomicAdd(&flags[F_MED_COUNT], 1u)] = (int32_t)row;
        }
    }
}

// Rows of kSmallRow+1 .. kScanRow entries (LIST = false) or the listed rows
// of kScanRow+1 .. kRegRow entries (LIST = true), sorted + uniqued in place
// in registers, a wave per row.  Without the list a wave scans `span`
// consecutive rows at a time (one lane each; no list, so no contended
// counter) and sorts the ones in range one after the other; the host picks
// span so that the grid's waves share the rows (a small graph gets one row
// per wave).  The longer rows take a list so that they spread over the
// waves, and an instantiation of their own so that the scan's register
// count stays low.  The rare longest rows get the bitmap sorter.
template <bool LIST>
__global__ void __launch_bounds__(kBlock) k_sort_rows(const int32_t *__restrict__ raw_off,
                                                      int32_t *raw_adj, int32_t n, int32_t span,
                                                      int32_t *ucnt, const int32_t *med_list,
                                                      const uint32_t *flags) {
    const int lane = lane_id();
    const int64_t wave0 = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
    const int64_t nitems = LIST ? (int64_t)flags[F_MED_COUNT] : ((int64_t)n + span - 1) / span;
    for (int64_t it = wave0; it < nitems; it += nwaves) {
        const int64_t c0 = it * span;
        uint64_t todo = 1ull;
        if (!LIST) {
            const int64_t mine = c0 + lane;
            const int32_t Lm = lane < span && mine < n ? raw_off[mine + 1] - raw_off[mine] : 0;
            todo = __ballot(Lm > kSmallRow && Lm <= kScanRow);
        }
        while (todo) {
            const int32_t row = LIST ? med_list[it] : (int32_t)(c0 + __builtin_ctzll(todo));
            todo &= todo - 1ull;
            const int32_t s = raw_off[row];
            const int32_t L = raw_off[row + 1] - s;
            int32_t *r = raw_adj + s;
            int32_t c;
            if (LIST) {
                if (L > 1024) c = wave_sort_row_regs<32>(r, L);
                else c = wave_sort_row_regs<16>(r, L);
            } else {
                if (L > 256) c = wave_sort_row_regs<8>(r, L);
                else if (L > 128) c = wave_sort_row_regs<4>(r, L);
                else if (L > 64) c = wave_sort_row_regs<2>(r, L);
                else c = wave_sort_row_regs<1>(r, L);
            }
            if (lane == 0) ucnt[row] = c;
        }
    }
}

// Rows per scan of k_sort_rows: all 64 lanes once the rows outnumber the
// grid's waves 64 to 1, fewer (down to one) below.
int32_t sort_span(int32_t n) {
    const int64_t waves = (int64_t)cu_count() * 16 * kWavesPerBlock;
    return (int32_t)std::max<int64_t>(1, std::min<int64_t>(kWave, ((int64_t)n + waves - 1) / waves));
}

// One workgroup per long row: set one bit per entry in a bitmap over the
// id range, then read the set bits back in ascending order.
__global__ void __launch_bounds__(kBlock) k_sort_big_rows(const int32_t *__restrict__ raw_off,
                                                          int32_t *raw_adj, int32_t *ucnt,
                                                          const int32_t *big_list,
                                                          const uint32_t *flags,
                                                          uint32_t *bitmaps, int64_t words) {
    __shared__ int64_t sh[kWavesPerBlock + 1];
    uint32_t *bm = bitmaps + (int64_t)blockIdx.x * words;
    const uint32_t nbig = flags[F_BIG_COUNT];
    for (uint32_t b = blockIdx.x; b < nbig; b += gridDim.x) {
        const int32_t row = big_list[b];
        const int32_t s = raw_off[row];
        const int32_t L = raw_off[row + 1] - s;
        int32_t *r = raw_adj + s;
        for (int64_t w = threadIdx.x; w < words; w += kBlock) bm[w] = 0u;
        __syncthreads();
        for (int32_t i = threadIdx.x; i < L; i += kBlock) {
            uint32_t x = (uint32_t)r[i];
            atomicOr(&bm[x >> 5], 1u << (x & 31));
        }
        __syncthreads();
        int64_t running = 0;
        for (int64_t w0 = 0; w0 < words; w0 += kBlock) {
            int64_t w = w0 + threadIdx.x;
            uint32_t word = w < words ? bm[w] : 0u;
            int64_t c = __popc(word);
            // block exclusive scan of c
            const int lanew = threadIdx.x & 63, wid = threadIdx.x >> 6;
            int64_t inc = wave_incl_scan(c);
            if (lanew == 63) sh[wid] = inc;
            __syncthreads();
            int64_t before = 0, total = 0;
            for (int q = 0; q < kWavesPerBlock; q++) {
                if (q < wid) before += sh[q];
                total += sh[q];
            }
            int64_t pos = running + before + inc - c;
            while (word) {
                int bit = __builtin_ctz(word);
                word &= word - 1;
                r[pos++] = (int32_t)(w * 32 + bit);
            }
            running += total;
            __syncthreads();
        }
        if (threadIdx.x == 0) ucnt[row] = (int32_t)running;
        __syncthreads();
    }
}

// The same with the bitmap in LDS (n <= kLdsBitmapIds): one workgroup of
// kBigNT threads per CU; clearing and scanning the bitmap stay on chip.
constexpr int kBigNT = 1024;
constexpr int64_t kLdsBitmapIds = 150 * 1024 * 8;   // 150 KiB of bits

__global__ void __launch_bounds__(kBigNT) k_sort_big_rows_lds(const int32_t *__restrict__ raw_off,
                                                              int32_t *raw_adj, int32_t *ucnt,
                                                              const int32_t *big_list,
                                                              const uint32_t *flags,
                                                              int32_t words) {
    extern __shared__ uint32_t bm[];
    __shared__ int32_t sh[kBigNT / kWave];
    constexpr int NW = kBigNT / kWave;
    const int tid = threadIdx.x, lanew = tid & 63, wid = tid >> 6;
    const uint32_t nbig = flags[F_BIG_COUNT];
    for (uint32_t b = blockIdx.x; b < nbig; b += gridDim.x) {
        const int32_t row = big_list[b];
        const int32_t s = raw_off[row];
        const int32_t L = raw_off[row + 1] - s;
        int32_t *r = raw_adj + s;
        for (int32_t w = tid; w < words; w += kBigNT) bm[w] = 0u;
        __syncthreads();
        for (int32_t i = tid; i < L; i += kBigNT) {
            const uint32_t x = (uint32_t)r[i];
            atomicOr(&bm[x >> 5], 1u << (x & 31));
        }
        __syncthreads();
        int32_t running = 0;
        for (int32_t w0 = 0; w0 < words; w0 += kBigNT) {
            const int32_t w = w0 + tid;
            uint32_t word = w < words ? bm[w] : 0u;
            const int32_t c = __popc(word);
            const int32_t inc = wave_incl_scan(c);
            if (lanew == 63) sh[wid] = inc;
            __syncthreads();
            int32_t before = 0, total = 0;
#pragma unroll
            for (int q = 0; q < NW; q++) {
                before += q < wid ? sh[q] : 0;
                total += sh[q];
            }
            int32_t pos = running + before + inc - c;
            while (word) {
                const int bit = __builtin_ctz(word);
                word &= word - 1;
                r[pos++] = w * 32 + bit;
            }
            running += total;
            __syncthreads();
        }
        if (tid == 0) ucnt[row] = running;
        __syncthreads();
    }
}

// Copies the unique rows into the final CSR and counts each vertex's arcs
// in the degree order (degrees are the unique counts); keep[i] records
// whether arc i points up in that order, so the fill does not look the
// degrees up again.
__global__ void __launch_bounds__(kBlock) k_compact_rows(const int32_t *__restrict__ raw_off,
                                                         const int32_t *__restrict__ raw_adj,
                                                         const int32_t *__restrict__ off,
                                                         const int32_t *__restrict__ deg,
                                                         int32_t *adj, int32_t n,
                                                         int32_t *outcnt, uint8_t *keep,
                                                         uint32_t *flags) {
    const int lane = lane_id(), gl = lane & (kSmallRow - 1), grp = lane / kSmallRow;
    const int64_t wave0 = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
    constexpr int kRows = kWave / kSmallRow;
    int32_t maxd = 0, big16 = 0;
    // 4 rows per wave: rows of <= 16 entries by a 16-lane group each, longer
    // ones by the whole wave after them
    for (int64_t r0 = wave0 * kRows; r0 < n; r0 += nwaves * kRows) {
        const int64_t row = r0 + grp;
        const bool live = row < n;
        const int32_t u = (int32_t)row;
        const int32_t src = live ? raw_off[row] : 0, dst = live ? off[row] : 0;
        const int32_t L = live ? off[row + 1] - dst : 0;
        maxd = L > maxd ? L : maxd;
        big16 += (gl == 0 && L > 65535) ? 1 : 0;
        const bool small = L <= kSmallRow;
        int32_t c = 0;
        if (small && gl < L) {
            const int32_t v = raw_adj[src + gl];
            adj[dst + gl] = v;
            c = rank_less(L, u, deg[v], v) ? 1 : 0;
            keep[dst + gl] = (uint8_t)c;
        }
#pragma unroll
        for (int o = kSmallRow / 2; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
        if (live && small && gl == 0) outcnt[u] = c;
        uint64_t longm = __ballot(live && !small && gl == 0);
        while (longm) {
            const int g = __builtin_ctzll(longm) / kSmallRow;
            longm &= longm - 1ull;
            const int32_t w = (int32_t)(r0 + g);
            const int32_t ws = raw_off[w], wd = off[w], wl = off[w + 1] - wd;
            int32_t cw = 0;
            for (int32_t i = lane; i < wl; i += kWave) {
                const int32_t v = raw_adj[ws + i];
                adj[wd + i] = v;
                const int32_t up = rank_less(wl, w, deg[v], v) ? 1 : 0;
                keep[wd + i] = (uint8_t)up;
                cw += up;
            }
            cw = wave_sum(cw);
            if (lane == 0) outcnt[w] = cw;
        }
    }
    maxd = wave_max(maxd);
    if (lane == 0 && maxd > 0) atomicMax(&flags[F_MAX_DEG], (uint32_t)maxd);
    big16 = wave_sum(big16);
    if (lane == 0 && big16 > 0) atomicAdd(&flags[F_DEG16], (uint32_t)big16);
}

__global__ void __launch_bounds__(kBlock) k_orient_count(const int32_t *__restrict__ off,
                                                         const int32_t *__restrict__ adj,
                                                         int32_t n, int32_t *outcnt,
                                                         uint8_t *keep) {
    const int lane = lane_id();
    const int64_t wave0 = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
    for (int64_t row = wave0; row < n; row += nwaves) {
        const int32_t u = (int32_t)row;
        const int32_t s = off[u], du = off[u + 1] - s;
        int32_t c = 0;
        for (int32_t i = lane; i < du; i += kWave) {
            int32_t v = adj[s + i];
            int32_t dv = off[v + 1] - off[v];
            const int32_t up = rank_less(du, u, dv, v) ? 1 : 0;
            keep[s + i] = (uint8_t)up;
            c += up;
        }
        c = wave_sum(c);
        if (lane == 0) outcnt[u] = c;
    }
}

__global__ void __launch_bounds__(kBlock) k_orient_fill(const int32_t *__restrict__ off,
                                                        const int32_t *__restrict__ adj,
                                                        const uint8_t *__restrict__ up,
                                                        const int32_t *__restrict__ dag_off,
                                                        int32_t n, int64_t cap, int32_t *dag_adj,
                                                        int32_t *dag_src, uint32_t *flags) {
    const int lane = lane_id(), gl = lane & (kSmallRow - 1), grp = lane / kSmallRow;
    const int64_t wave0 = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
    constexpr int kRows = kWave / kSmallRow;
    int32_t maxo = 0;
    // 4 rows per wave: rows of <= 16 entries by a 16-lane group each, longer
    // ones by the whole wave after them
    for (int64_t r0 = wave0 * kRows; r0 < n; r0 += nwaves * kRows) {
        const int64_t row = r0 + grp;
        const bool live = row < n;
        const int32_t su = live ? off[row] : 0, dsu = live ? off[row + 1] - su : 0;
        const bool small = dsu <= kSmallRow;
        int32_t v = 0;
        bool keep = false;
        if (small && gl < dsu) {
            v = adj[su + gl];
            keep = up[su + gl] != 0;
        }
        const uint32_t gmask =
            (uint32_t)(__ballot(keep) >> (grp * kSmallRow)) & ((1u << kSmallRow) - 1u);
        if (keep) {
            const int32_t p = dag_off[row] + __popc(gmask & ((1u << gl) - 1u));
            if (p < cap) {
                dag_adj[p] = v;
                dag_src[p] = (int32_t)row;
            } else {
                atomicOr(&flags[F_ERR], 4u);   // more arcs than the storage holds
            }
        }
        maxo = max(maxo, __popc(gmask));
        uint64_t longm = __ballot(live && !small && gl == 0);
        while (longm) {
            const int32_t u = (int32_t)(r0 + __builtin_ctzll(longm) / kSmallRow);
            longm &= longm - 1ull;
            const int32_t s = off[u], du = off[u + 1] - s;
            int32_t base = dag_off[u];
            for (int32_t i0 = 0; i0 < du; i0 += kWave) {
                int32_t i = i0 + lane;
                int32_t v = i < du ? adj[s + i] : 0;
                bool keep = false;
                if (i < du) keep = up[s + i] != 0;
                uint64_t mask = __ballot(keep);
                if (keep) {
                    int32_t p = base + lanes_below(mask);
                    if (p < cap) {
                        dag_adj[p] = v;
                        dag_src[p] = u;
                    } else {
                        atomicOr(&flags[F_ERR], 4u);   // more arcs than the storage holds
                    }
                }
                base += __popcll(mask);
            }
            int32_t d = base - dag_off[u];
            maxo = d > maxo ? d : maxo;
        }
    }
    maxo = wave_max(maxo);
    if (lane == 0 && maxo > 0) atomicMax(&flags[F_MAX_OUT], (uint32_t)maxo);
}

// Orientation key of the degree order, key[v] = deg(v): the local-graph
// kernels rank each root's out-neighbours by (key, id), as the DAG does.
__global__ void k_degree_key(const int32_t *__restrict__ off, int32_t n, int32_t *key) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        key[v] = off[v + 1] - off[v];
}

__global__ void k_meta(const int32_t *off, const int32_t *dag_off, int32_t n,
                       const uint32_t *flags, int64_t *meta) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        meta[0] = off[n];
        meta[1] = dag_off[n];
        meta[2] = flags[F_MAX_DEG];
        meta[3] = flags[F_MAX_OUT];
        meta[4] = flags[F_ERR];
        meta[5] = flags[F_BIG_COUNT];
        meta[6] = flags[F_DEG16];
    }
}

// Checks of a caller's CSR (one wave per row).  Always: offsets ascending
// and within [0, nnz], ids in [0, n); with FULL also strictly ascending rows,
// no self-loop, and every arc (u, w) matched by (w, u).  Any failure sets
// F_ERR; the largest degree goes to F_MAX_DEG.
template <bool FULL>
__global__ void __launch_bounds__(kBlock) k_check_csr(const int32_t *__restrict__ off,
                                                      const int32_t *__restrict__ adj, int32_t n,
                                                      int64_t nnz, uint32_t *flags) {
    const int lane = lane_id();
    const int64_t wave0 = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
    if (blockIdx.x == 0 && threadIdx.x == 0 && (off[0] != 0 || (int64_t)off[n] != nnz))
        atomicOr(&flags[F_ERR], 2u);
    int32_t maxd = 0, big16 = 0;
    for (int64_t row = wave0; row < n; row += nwaves) {
        const int32_t u = (int32_t)row;
        const int32_t s = off[u], e = off[u + 1];
        if (s < 0 || e < s || (int64_t)e > nnz) {
            if (lane == 0) atomicOr(&flags[F_ERR], 2u);
            continue;
        }
        maxd = max(maxd, e - s);
        big16 += (lane == 0 && e - s > 65535) ? 1 : 0;
        bool bad = false;
        for (int32_t i = s + lane; i < e; i += kWave) {
            const int32_t w = adj[i];
            if (w < 0 || w >= n) {
                bad = true;
                continue;
            }
            if (FULL) {
                if (w == u || (i > s && adj[i - 1] >= w)) bad = true;
                // (w, u) present: binary search u in N(w), whose bounds are
                // checked first
                const int32_t ws = off[w], we = off[w + 1];
                if (ws < 0 || we < ws || (int64_t)we > nnz) {
                    bad = true;
                    continue;
                }
                int32_t lo = ws, hi = we;
                while (lo < hi) {
                    const int32_t mid = (lo + hi) >> 1;
                    if (adj[mid] < u) lo = mid + 1; else hi = mid;
                }
                if (lo >= we || adj[lo] != u) bad = true;
            }
        }
        if (__any(bad) && lane == 0) atomicOr(&flags[F_ERR], 2u);
    }
    maxd = wave_max(maxd);
    if (lane == 0 && maxd > 0) atomicMax(&flags[F_MAX_DEG], (uint32_t)maxd);
    big16 = wave_sum(big16);
    if (lane == 0 && big16 > 0) atomicAdd(&flags[F_DEG16], (uint32_t)big16);
}

struct BuildLayout {
    // graph storage
    int32_t *off, *adj, *dag_off, *dag_adj, *dag_src;
    int64_t *meta;
    int32_t *okey;
    // scratch
    int32_t *cnt, *raw_off, *raw_adj, *ucnt, *outcnt, *big_list, *med_list;
    uint8_t *keep;                                  // per final arc: points up in the order
    int32_t S, nb;                                  // buckets of 2^S source ids (S = 0: none)
    int32_t *bucket_cnt, *bucket_off, *bucket_cur, *bsrc, *bdst;
    int64_t *scan_tmp;
    uint32_t *flags, *bitmaps;
    int64_t words;
    int nbig_blocks;
    uint64_t graph_bytes, scratch_bytes;
};

// Bucket shift for n vertices: the smallest S >= 10 with at most
// kTargetBuckets buckets of 2^S ids, or 0 when 2^S would exceed
// kMaxBucketIds.  About 1024 buckets (4 per CU at 256 CUs) keep a bucket
// that holds a hub's arcs from dominating the per-bucket pass.
constexpr int kTargetBuckets = 1024;
int32_t bucket_shift(int32_t n) {
    int32_t S = 10;
    while (((int64_t)n + (1ll << S) - 1) >> S > kTargetBuckets) S++;
    return (1 << S) <= kMaxBucketIds ? S : 0;
}

BuildLayout layout(int32_t n, int64_t E, void *gmem, void *smem) {
    BuildLayout L{};
    Carve g(gmem, ~0ull);
    L.off = g.take<int32_t>((uint64_t)n + 1);
    L.adj = g.take<int32_t>((uint64_t)(2 * E));
    L.dag_off = g.take<int32_t>((uint64_t)n + 1);
    L.dag_adj = g.take<int32_t>((uint64_t)E);
    L.dag_src = g.take<int32_t>((uint64_t)E);
    L.meta = g.take<int64_t>(8);
    L.okey = g.take<int32_t>((uint64_t)n + 1);
    L.graph_bytes = g.used;
    Carve s(smem, ~0ull);
    L.cnt = s.take<int32_t>((uint64_t)n + 1);
    L.raw_off = s.take<int32_t>((uint64_t)n + 1);
    L.raw_adj = s.take<int32_t>((uint64_t)(2 * E));
    L.ucnt = s.take<int32_t>((uint64_t)n + 1);
    L.outcnt = s.take<int32_t>((uint64_t)n + 1);
    L.big_list = s.take<int32_t>((uint64_t)n + 1);
    L.med_list = s.take<int32_t>((uint64_t)n + 1);
    L.keep = s.take<uint8_t>((uint64_t)(2 * E));
    L.scan_tmp = s.take<int64_t>(scan_tmp_words((uint64_t)n + 1));
    L.flags = s.take<uint32_t>(F_WORDS);
    L.S = bucket_shift(n);
    if (L.S > 0) {
        L.nb = (int32_t)(((int64_t)n + (1ll << L.S) - 1) >> L.S);
        L.bucket_cnt = s.take<int32_t>((uint64_t)L.nb + 1);
        L.bucket_off = s.take<int32_t>((uint64_t)L.nb + 1);
        L.bucket_cur = s.take<int32_t>((uint64_t)L.nb + 1);
        L.bsrc = s.take<int32_t>((uint64_t)(2 * E));
        L.bdst = s.take<int32_t>((uint64_t)(2 * E));
    }
    L.words = ((int64_t)n + 31) / 32;
    // bitmap sorters: as many concurrent workgroups as fit in 64 MiB, 1..256
    int64_t per = L.words * 4;
    int64_t nb = (64ll << 20) / (per > 0 ? per : 1);
    L.nbig_blocks = (int)std::max<int64_t>(1, std::min<int64_t>(256, nb));
    L.bitmaps = s.take<uint32_t>((uint64_t)L.words * L.nbig_blocks);
    L.scratch_bytes = s.used;
    return L;
}

unsigned wave_grid(int64_t rows) {
    int64_t blocks = (rows + kWavesPerBlock - 1) / kWavesPerBlock;
    int64_t cap = (int64_t)cu_count() * 16;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(blocks, cap));
}

unsigned flat_grid(int64_t items) {
    int64_t blocks = (items + kBlock - 1) / kBlock;
    int64_t cap = (int64_t)cu_count() * 32;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(blocks, cap));
}

}  // namespace

hipError_t degree_key(const int32_t *off, int32_t n, int32_t *key, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)std::min<int64_t>(((int64_t)n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_degree_key, dim3(blocks), dim3(256), 0, st, off, n, key);
    return hipGetLastError();
}

static gpm_status enqueue_build(int32_t n, const int32_t *d_u, const int32_t *d_v, int64_t E,
                                const BuildLayout &L, hipStream_t st);

gpm_status graph_build_bytes(int32_t n, int64_t E, uint64_t *gb, uint64_t *sb) {
    if (n < 1 || n > INT32_MAX - 1) return fail(GPM_INVALID_ARGUMENT, "n must be in [1, 2^31-2]");
    if (E < 0 || 2 * E >= (int64_t)INT32_MAX)
        return fail(GPM_UNSUPPORTED, "2 * n_input_edges must be below 2^31");
    BuildLayout L = layout(n, E, nullptr, nullptr);
    *gb = L.graph_bytes;
    *sb = L.scratch_bytes;
    return GPM_OK;
}

gpm_status graph_build(int32_t n, const int32_t *d_u, const int32_t *d_v, int64_t E, void *gmem,
                       uint64_t gbytes, void *smem, uint64_t sbytes, hipStream_t st,
                       gpm_graph **out) {
    uint64_t need_g, need_s;
    gpm_status rc = graph_build_bytes(n, E, &need_g, &need_s);
    if (rc != GPM_OK) return rc;
    if (!out) return fail(GPM_INVALID_ARGUMENT, "out is NULL");
    if (E > 0 && (!d_u || !d_v)) return fail(GPM_INVALID_ARGUMENT, "edge arrays are NULL");
    if (!gmem || !smem) return fail(GPM_INVALID_ARGUMENT, "graph or scratch memory is NULL");
    if (((uintptr_t)gmem & 255) || ((uintptr_t)smem & 255))
        return fail(GPM_INVALID_ARGUMENT, "device buffers must be 256-byte aligned");
    if (gbytes < need_g || sbytes < need_s)
        return fail(GPM_OUT_OF_MEMORY, "graph or scratch buffer smaller than gpm_graph_build_bytes");
    BuildLayout L = layout(n, E, gmem, smem);
    gpm_status rc2 = enqueue_build(n, d_u, d_v, E, L, st);
    if (rc2 != GPM_OK) return rc2;

    int64_t meta[8] = {0};
    GPM_HIP(hipMemcpyAsync(meta, L.meta, sizeof(int64_t) * 7, hipMemcpyDeviceToHost, st));
    GPM_HIP(hipStreamSynchronize(st));
    if (meta[4] != 0) return fail(GPM_NOT_CANONICAL, "an input vertex id is outside [0, n)");
    if (meta[0] % 2 != 0 || meta[1] * 2 != meta[0])
        return fail(GPM_DEVICE_ERROR, "graph build produced inconsistent sizes");

    gpm_graph *g = new (std::nothrow) gpm_graph;
    if (!g) return fail(GPM_OUT_OF_MEMORY, "host allocation of the graph handle failed");
    g->n = n;
    g->m = meta[1];
    g->max_degree = (int32_t)meta[2];
    g->max_out_degree = (int32_t)meta[3];
    g->n_deg_over_65535 = (int32_t)meta[6];
    g->off = L.off;
    g->adj = L.adj;
    g->dag_off = L.dag_off;
    g->dag_adj = L.dag_adj;
    g->dag_src = L.dag_src;
    g->okey = L.okey;
    *out = g;
    return GPM_OK;
}

gpm_status graph_from_csr_bytes(int32_t n, int64_t nnz, uint64_t *gb, uint64_t *sb) {
    if (n < 1 || n > INT32_MAX - 1) return fail(GPM_INVALID_ARGUMENT, "n must be in [1, 2^31-2]");
    if (nnz < 0 || (nnz & 1) || nnz >= (int64_t)INT32_MAX)
        return fail(GPM_UNSUPPORTED, "nnz must be even and below 2^31");
    BuildLayout L = layout(n, nnz / 2, nullptr, nullptr);
    *gb = L.graph_bytes;
    Carve s(nullptr, ~0ull);
    s.take<int32_t>((uint64_t)n + 1);                              // out-degrees
    s.take<int64_t>(scan_tmp_words((uint64_t)n + 1));
    s.take<uint32_t>(F_WORDS);
    s.take<uint8_t>((uint64_t)nnz);                                // arc points up
    *sb = s.used;
    return GPM_OK;
}

gpm_status graph_from_csr(int32_t n, const int32_t *d_off, const int32_t *d_adj, int64_t nnz,
                          int32_t validate, void *gmem, uint64_t gbytes, void *smem,
                          uint64_t sbytes, hipStream_t st, gpm_graph **out) {
    uint64_t need_g, need_s;
    gpm_status rc = graph_from_csr_bytes(n, nnz, &need_g, &need_s);
    if (rc != GPM_OK) return rc;
    if (!out) return fail(GPM_INVALID_ARGUMENT, "out is NULL");
    if (!d_off || (nnz > 0 && !d_adj)) return fail(GPM_INVALID_ARGUMENT, "CSR arrays are NULL");
    if (!gmem || !smem) return fail(GPM_INVALID_ARGUMENT, "graph or scratch memory is NULL");
    if (((uintptr_t)gmem & 255) || ((uintptr_t)smem & 255))
        return fail(GPM_INVALID_ARGUMENT, "device buffers must be 256-byte aligned");
    if (gbytes < need_g || sbytes < need_s)
        return fail(GPM_OUT_OF_MEMORY, "graph or scratch buffer smaller than required");
    BuildLayout L = layout(n, nnz / 2, gmem, nullptr);
    Carve sc(smem, ~0ull);
    int32_t *outcnt = sc.take<int32_t>((uint64_t)n + 1);
    int64_t *scan_tmp = sc.take<int64_t>(scan_tmp_words((uint64_t)n + 1));
    uint32_t *flags = sc.take<uint32_t>(F_WORDS);
    uint8_t *up = sc.take<uint8_t>((uint64_t)nnz);
    {
        Span whole("graph_from_csr", st);
        GPM_HIP(fill_u32(flags, 0, F_WORDS, st));
        GPM_HIP(hipMemcpyAsync(L.off, d_off, sizeof(int32_t) * ((size_t)n + 1),
                               hipMemcpyDeviceToDevice, st));
        if (nnz > 0)
            GPM_HIP(hipMemcpyAsync(L.adj, d_adj, sizeof(int32_t) * (size_t)nnz,
                                   hipMemcpyDeviceToDevice, st));
        if (validate)
            hipLaunchKernelGGL(k_check_csr<true>, dim3(wave_grid(n)), dim3(kBlock), 0, st, L.off,
                               L.adj, n, nnz, flags);
        else
            hipLaunchKernelGGL(k_check_csr<false>, dim3(wave_grid(n)), dim3(kBlock), 0, st,
                               L.off, L.adj, n, nnz, flags);
        GPM_LAUNCH_CHECK("k_check_csr");
        // orientation needs a valid CSR: read the check result first
        int64_t meta[8] = {0};
        hipLaunchKernelGGL(k_meta, dim3(1), dim3(64), 0, st, L.off, L.off, n, flags, L.meta);
        GPM_HIP(hipMemcpyAsync(meta, L.meta, sizeof(int64_t) * 7, hipMemcpyDeviceToHost, st));
        GPM_HIP(hipStreamSynchronize(st));
        if (meta[4] != 0) return fail(GPM_NOT_CANONICAL, "the CSR is not in canonical form");
        hipLaunchKernelGGL(k_orient_count, dim3(wave_grid(n)), dim3(kBlock), 0, st, L.off, L.adj,
                           n, outcnt, up);
        GPM_LAUNCH_CHECK("k_orient_count");
        GPM_HIP(exclusive_scan_i32(outcnt, L.dag_off, (uint64_t)n, scan_tmp, st));
        hipLaunchKernelGGL(k_orient_fill, dim3(wave_grid(n)), dim3(kBlock), 0, st, L.off, L.adj,
                           up, L.dag_off, n, nnz / 2, L.dag_adj, L.dag_src, flags);
        GPM_LAUNCH_CHECK("k_orient_fill");
        GPM_HIP(degree_key(L.off, n, L.okey, st));
        hipLaunchKernelGGL(k_meta, dim3(1), dim3(64), 0, st, L.off, L.dag_off, n, flags, L.meta);
        GPM_LAUNCH_CHECK("k_meta");
    }
    int64_t meta[8] = {0};
    GPM_HIP(hipMemcpyAsync(meta, L.meta, sizeof(int64_t) * 7, hipMemcpyDeviceToHost, st));
    GPM_HIP(hipStreamSynchronize(st));
    if (meta[4] != 0 || meta[0] != nnz || meta[1] * 2 != meta[0])
        return fail(GPM_NOT_CANONICAL, "the CSR is not symmetric");
    gpm_graph *g = new (std::nothrow) gpm_graph;
    if (!g) return fail(GPM_OUT_OF_MEMORY, "host allocation of the graph handle failed");
    g->n = n;
    g->m = meta[1];
    g->max_degree = (int32_t)meta[2];
    g->max_out_degree = (int32_t)meta[3];
    g->n_deg_over_65535 = (int32_t)meta[6];
    g->off = L.off;
    g->adj = L.adj;
    g->dag_off = L.dag_off;
    g->dag_adj = L.dag_adj;
    g->dag_src = L.dag_src;
    g->okey = L.okey;
    *out = g;
    return GPM_OK;
}

// All build kernels, in stream order (a1 then a2).
static gpm_status enqueue_build(int32_t n, const int32_t *d_u, const int32_t *d_v, int64_t E,
                         const BuildLayout &L, hipStream_t st) {
    Span whole("graph_build", st);
    GPM_HIP(fill_u32(L.flags, 0, F_WORDS, st));
    if (E > 0 && L.S > 0) {
        const int64_t tiles = (E + kTileEdges - 1) / kTileEdges;
        const unsigned tgrid = (unsigned)std::min<int64_t>(tiles, (int64_t)cu_count() * 8);
        GPM_HIP(fill_u32(L.bucket_cnt, 0, (uint64_t)L.nb + 1, st));
        hipLaunchKernelGGL(k_bucket_count, dim3(tgrid), dim3(kBlock), 0, st, d_u, d_v, E, n, L.S,
                           L.nb, L.bucket_cnt, L.flags);
        GPM_LAUNCH_CHECK("k_bucket_count");
        GPM_HIP(exclusive_scan_i32(L.bucket_cnt, L.bucket_off, (uint64_t)L.nb, L.scan_tmp, st));
        GPM_HIP(hipMemcpyAsync(L.bucket_cur, L.bucket_off, sizeof(int32_t) * (size_t)L.nb,
                               hipMemcpyDeviceToDevice, st));
        // the largest tile (up to kTileEdges, a multiple of 1024) whose arcs
        // fit in LDS next to the bucket tables
        int32_t te = kTileEdges;
        while (te > 1024 && scatter_lds_bytes(L.nb, te) > (size_t)150 * 1024) te -= 1024;
        const int64_t stiles = (E + te - 1) / te;
        hipLaunchKernelGGL(k_bucket_scatter,
                           dim3((unsigned)std::min<int64_t>(stiles, (int64_t)cu_count())),
                           dim3(kScatterNT), scatter_lds_bytes(L.nb, te), st, d_u, d_v, E, n,
                           L.S, L.nb, te, L.bucket_cur, L.bsrc, L.bdst);
        GPM_LAUNCH_CHECK("k_bucket_scatter");
        hipLaunchKernelGGL(k_bucket_rows,
                           dim3((unsigned)std::min<int64_t>(L.nb, (int64_t)cu_count() * 2)),
                           dim3(kBucketNT), 0, st, L.bucket_off, L.bsrc, L.bdst, n, L.S, L.nb,
                           L.raw_off, L.raw_adj);
        GPM_LAUNCH_CHECK("k_bucket_rows");
    } else {
        GPM_HIP(fill_u32(L.cnt, 0, (uint64_t)n + 1, st));
        if (E > 0) {
            hipLaunchKernelGGL(k_count_raw, dim3(flat_grid(E)), dim3(kBlock), 0, st, d_u, d_v, E,
                               n, L.cnt, L.flags);
            GPM_LAUNCH_CHECK("k_count_raw");
        }
        GPM_HIP(exclusive_scan_i32(L.cnt, L.raw_off, (uint64_t)n, L.scan_tmp, st));
        GPM_HIP(fill_u32(L.cnt, 0, (uint64_t)n + 1, st));
        if (E > 0) {
            hipLaunchKernelGGL(k_scatter_raw, dim3(flat_grid(E)), dim3(kBlock), 0, st, d_u, d_v,
                               E, n, L.raw_off, L.cnt, L.raw_adj);
            GPM_LAUNCH_CHECK("k_scatter_raw");
        }
    }
    hipLaunchKernelGGL(k_sort_small_rows, dim3(wave_grid(((int64_t)n + 3) / 4)), dim3(kBlock), 0,
                       st, L.raw_off, L.raw_adj, n, L.ucnt, L.med_list, L.big_list, L.flags);
    GPM_LAUNCH_CHECK("k_sort_small_rows");
    {
        const int32_t span = sort_span(n);
        hipLaunchKernelGGL(k_sort_rows<false>, dim3(wave_grid(((int64_t)n + span - 1) / span)),
                           dim3(kBlock), 0, st, L.raw_off, L.raw_adj, n, span, L.ucnt, nullptr,
                           L.flags);
        hipLaunchKernelGGL(k_sort_rows<true>, dim3(wave_grid(n)), dim3(kBlock), 0, st, L.raw_off,
                           L.raw_adj, n, 1, L.ucnt, L.med_list, L.flags);
    }
    GPM_LAUNCH_CHECK("k_sort_rows");
    if (n <= kLdsBitmapIds)
        hipLaunchKernelGGL(k_sort_big_rows_lds, dim3((unsigned)cu_count()), dim3(kBigNT),
                           (size_t)L.words * 4, st, L.raw_off, L.raw_adj, L.ucnt, L.big_list,
                           L.flags, (int32_t)L.words);
    else
        hipLaunchKernelGGL(k_sort_big_rows, dim3(L.nbig_blocks), dim3(kBlock), 0, st, L.raw_off,
                           L.raw_adj, L.ucnt, L.big_list, L.flags, L.bitmaps, L.words);
    GPM_LAUNCH_CHECK("k_sort_big_rows");
    GPM_HIP(exclusive_scan_i32(L.ucnt, L.off, (uint64_t)n, L.scan_tmp, st));
    hipLaunchKernelGGL(k_compact_rows, dim3(wave_grid(n)), dim3(kBlock), 0, st, L.raw_off,
                       L.raw_adj, L.off, L.ucnt, L.adj, n, L.outcnt, L.keep, L.flags);
    GPM_LAUNCH_CHECK("k_compact_rows");
    GPM_HIP(exclusive_scan_i32(L.outcnt, L.dag_off, (uint64_t)n, L.scan_tmp, st));
    hipLaunchKernelGGL(k_orient_fill, dim3(wave_grid(n)), dim3(kBlock), 0, st, L.off, L.adj,
                       L.keep, L.dag_off, n, E, L.dag_adj, L.dag_src, L.flags);
    GPM_LAUNCH_CHECK("k_orient_fill");
    GPM_HIP(degree_key(L.off, n, L.okey, st));
    hipLaunchKernelGGL(k_meta, dim3(1), dim3(64), 0, st, L.off, L.dag_off, n, L.flags, L.meta);
    GPM_LAUNCH_CHECK("k_meta");
    return GPM_OK;
}

// Sorting the rows of any CSR in place with the build's sorters (rows of
// distinct ids in [0, n) stay whole; duplicates would be dropped and counted
// out in ucnt).  The work area: counts, the two row lists, the flags and
// the bitmap sorters' bitmaps.
struct RowSortArea {
    int32_t *ucnt, *big_list, *med_list;
    uint32_t *flags, *bitmaps;
    int64_t words;
    int nbig_blocks;
};

RowSortArea row_sort_layout(int32_t n, void *base, uint64_t *bytes) {
    RowSortArea A{};
    Carve c(base, ~0ull);
    A.ucnt = c.take<int32_t>((uint64_t)n + 1);
    A.big_list = c.take<int32_t>((uint64_t)n + 1);
    A.med_list = c.take<int32_t>((uint64_t)n + 1);
    A.flags = c.take<uint32_t>(F_WORDS);
    A.words = ((int64_t)n + 31) / 32;
    const int64_t per = A.words * 4;
    const int64_t nb = (64ll << 20) / (per > 0 ? per : 1);
    A.nbig_blocks = (int)std::max<int64_t>(1, std::min<int64_t>(256, nb));
    A.bitmaps = c.take<uint32_t>((uint64_t)A.words * A.nbig_blocks);
    if (bytes) *bytes = c.used;
    return A;
}

uint64_t row_sort_bytes(int32_t n) {
    uint64_t b = 0;
    row_sort_layout(n, nullptr, &b);
    return b;
}

gpm_status sort_rows(const int32_t *off, int32_t *adj, int32_t n, void *area, hipStream_t st) {
    RowSortArea A = row_sort_layout(n, area, nullptr);
    GPM_HIP(fill_u32(A.flags, 0, F_WORDS, st));
    hipLaunchKernelGGL(k_sort_small_rows, dim3(wave_grid(((int64_t)n + 3) / 4)), dim3(kBlock), 0,
                       st, off, adj, n, A.ucnt, A.med_list, A.big_list, A.flags);
    const int32_t span = sort_span(n);
    hipLaunchKernelGGL(k_sort_rows<false>, dim3(wave_grid(((int64_t)n + span - 1) / span)),
                       dim3(kBlock), 0, st, off, adj, n, span, A.ucnt, nullptr, A.flags);
    hipLaunchKernelGGL(k_sort_rows<true>, dim3(wave_grid(n)), dim3(kBlock), 0, st, off, adj, n, 1,
                       A.ucnt, A.med_list, A.flags);
    if (n <= kLdsBitmapIds)
        hipLaunchKernelGGL(k_sort_big_rows_lds, dim3((unsigned)cu_count()), dim3(kBigNT),
                           (size_t)A.words * 4, st, off, adj, A.ucnt, A.big_list, A.flags,
                           (int32_t)A.words);
    else
        hipLaunchKernelGGL(k_sort_big_rows, dim3(A.nbig_blocks), dim3(kBlock), 0, st, off, adj,
                           A.ucnt, A.big_list, A.flags, A.bitmaps, A.words);
    GPM_LAUNCH_CHECK("sort_rows");
    return GPM_OK;
}

}  // namespace gpm
