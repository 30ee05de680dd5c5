// Core numbers and the core-value orientation (Appendix B.2 names two
// orientations for cliques: by degree and by core value).
//
// Core numbers as the fixed point of the h-index operator (Lu, Zhou, Zhang
// and Stanley, Nature Communications 2016; Montresor, De Pellegrini and
// Miorandi, 2013): starting from an upper bound (the degree, capped by the
// largest h with at least h + 1 vertices of degree >= h), every vertex
// repeatedly takes the h-index of its neighbours' values (the largest h such
// that at least h of them are >= h).  Values only decrease and settle at the
// core numbers.  Each round is one kernel over the vertices marked active:
// a vertex is evaluated when a neighbour's value dropped below its own in
// the previous round, updates in place, and marks the neighbours its drop
// can affect; the run ends after a round without a change.  The h-index of
// a vertex of degree <= 64 comes from ballots over its neighbours' values in
// registers, of a larger one from an LDS histogram of min(value, own value)
// (a wave's up to degree 512, a workgroup's above; at most 4096 bins, hence
// the cap on the bound).  RMAT-14/16/18 take 20,
// 29 and 59 rounds of the synchronous form against hundreds of peeling
// levels.  Graphs whose bound exceeds 4095 (or that would need more than
// kMaxRounds rounds) are peeled instead:
//
// Core numbers by level-synchronous peeling.  For level L = 0, 1, ...: every
// vertex not yet removed whose remaining degree is at most L is removed with
// core number L (a scan), and removing a vertex lowers its live neighbours'
// remaining degrees (atomic decrements); a neighbour whose degree falls from
// L + 1 to L is removed at the same level, in the next sub-round.  Each
// vertex is removed once, when the decrement that takes it to L is the one
// that sees L + 1, so the frontier lists never repeat a vertex.  Levels with
// nothing to remove are skipped by taking the smallest remaining degree.
//
// Scans and sub-rounds are steps of one kernel, k_core_step, queued back to
// back.  A step reads the peeling state (level, scan or sub-round, its
// input frontier's size) that the previous step left, does its share, and
// the last workgroup to finish (a count of finished workgroups) turns the
// step's counters into the next state; the kernel boundary orders the steps,
// so no workgroup ever waits for another.  The host queues steps in batches
// and reads the state once per batch; steps queued past the end do nothing.
// Scans walk a list of the vertices still live at the previous scan (all of
// them at the first) and write the ones they keep to a second list, so a
// scan costs the live vertices rather than n.
//
// Orientation: arc u -> v iff (key(u), u) < (key(v), v); each row's arcs
// keep ascending id order.  By degree, key = the degree (the build's
// orientation).  By core value, key = (core << S) | min(degree, 2^S - 1),
// S = 31 - bits(largest core): the core value first, then, among equal core
// values, the degree, so a hub does not point at its whole core (by core
// value and id alone, RMAT-20's largest out-degree is 1289; with the degree
// as second key 702, against 707 by degree and 639 for the degeneracy).
#include <algorithm>
#include <climits>
#include <cstdlib>
#include <mutex>

#include "gpm_internal.h"

namespace gpm {

namespace {

constexpr int kCoreBlock = 256;
constexpr int kCoreWaves = kCoreBlock / kWave;

// ctl words: the peeling state (level; mode; input frontier size and which
// frontier buffer holds it; live-list size and buffer; first scan; largest
// core so far), the finished-workgroup count, the step's counters (output
// size, smallest kept degree, vertices kept) and the orientation's largest
// out-degree
enum { S_LEVEL = 0, S_MODE = 1, S_CIN = 2, S_FBUF = 3, S_LIVE = 4, S_LBUF = 5, S_FIRST = 6,
       S_MAXCORE = 7, S_DONE = 8, K_CNT = 9, K_MIN = 10, K_KEPT = 11, C_MAX_OUT = 12,
       H_UB = 13, H_MAXC = 14, C_WORDS = 16 };
enum { M_SCAN = 0, M_PROCESS = 1, M_END = 2 };

__global__ void __launch_bounds__(kCoreBlock) k_core_init(const int32_t *__restrict__ off,
                                                          int32_t n, int32_t *deg,
                                                          int32_t *core) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        deg[v] = off[v + 1] - off[v];
        core[v] = -1;
    }
}

// One step of the peeling (see above).  F0/F1: frontier buffers (scans
// write F0, sub-rounds alternate); L0/L1: live lists.
__global__ void __launch_bounds__(kCoreBlock) k_core_step(const int32_t *__restrict__ off,
                                                          const int32_t *__restrict__ adj,
                                                          int32_t n, int32_t *deg, int32_t *core,
                                                          int32_t *F0, int32_t *F1, int32_t *L0,
                                                          int32_t *L1, uint32_t *ctl) {
    __shared__ int32_t wmin[kCoreWaves];
    const uint32_t mode = ctl[S_MODE];
    if (mode == M_END) return;
    const int32_t level = (int32_t)ctl[S_LEVEL];
    const int lane = lane_id();
    if (mode == M_SCAN) {
        // live vertices of remaining degree <= level into F0, the others to
        // the other live list; the smallest degree kept, for skipping levels
        const bool first = ctl[S_FIRST] != 0;
        const int64_t live = first ? (int64_t)n : (int64_t)ctl[S_LIVE];
        const int32_t *lin = ctl[S_LBUF] ? L1 : L0;
        int32_t *lout = ctl[S_LBUF] ? L0 : L1;
        const int64_t stride = (int64_t)gridDim.x * blockDim.x;
        int32_t mn = INT_MAX;
        for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < live; i0 += stride) {
            const int64_t i = i0 + threadIdx.x;
            int32_t v = -1;
            if (i < live) v = first ? (int32_t)i : lin[i];
            const bool alive = v >= 0 && core[v] < 0;
            const int32_t d = alive ? deg[v] : INT_MAX;
            const bool take = alive && d <= level;
            const bool keep = alive && !take;
            if (take) core[v] = level;
            else mn = min(mn, d);
            const uint64_t tmask = __ballot(take), kmask = __ballot(keep);
            if (tmask) {
                uint32_t base = 0;
                if (lane == 0) base = atomicAdd(ctl + K_CNT, (uint32_t)__popcll(tmask));
                base = __shfl(base, 0);
                if (take) F0[base + lanes_below(tmask)] = v;
            }
            if (kmask) {
                uint32_t base = 0;
                if (lane == 0) base = atomicAdd(ctl + K_KEPT, (uint32_t)__popcll(kmask));
                base = __shfl(base, 0);
                if (keep) lout[base + lanes_below(kmask)] = v;
            }
        }
        // one atomic per workgroup: a per-wave atomic on one word
        // serialises thousands of waves
        mn = -wave_max(-mn);
        if (lane == 0) wmin[threadIdx.x / kWave] = mn;
        __syncthreads();
        if (threadIdx.x == 0) {
            int32_t b = wmin[0];
            for (int w = 1; w < kCoreWaves; w++) b = min(b, wmin[w]);
            if (b != INT_MAX) atomicMin(ctl + K_MIN, (uint32_t)b);
        }
    } else {
        // one sub-round: a wave per removed vertex lowers its live
        // neighbours' degrees; those reaching the level are removed
        const int32_t *fin = ctl[S_FBUF] ? F1 : F0;
        int32_t *fout = ctl[S_FBUF] ? F0 : F1;
        const int64_t cin = (int64_t)ctl[S_CIN];
        const int64_t nwaves = (int64_t)gridDim.x * kCoreWaves;
        for (int64_t i = (int64_t)blockIdx.x * kCoreWaves + threadIdx.x / kWave; i < cin;
             i += nwaves) {
            const int32_t v = fin[i];
            const int32_t e = off[v + 1];
            for (int32_t j0 = off[v]; j0 < e; j0 += kWave) {
                const int32_t j = j0 + lane;
                bool app = false;
                int32_t u = 0;
                if (j < e) {
                    u = adj[j];
                    if (core[u] < 0) {
                        const int32_t old = atomicSub(deg + u, 1);
                        if (old == level + 1) {
                            core[u] = level;
                            app = true;
                        }
                    }
                }
                const uint64_t mask = __ballot(app);
                if (!mask) continue;
                uint32_t base = 0;
                if (lane == 0) base = atomicAdd(ctl + K_CNT, (uint32_t)__popcll(mask));
                base = __shfl(base, 0);
                if (app) fout[base + lanes_below(mask)] = u;
            }
        }
    }
    // the last workgroup to finish sets the next state (every workgroup has
    // read the current one by then) and clears the step's counters.  Only
    // the counters cross workgroups inside the step, and they are device
    // atomics: each workgroup's counter updates are complete (the barrier
    // waits for its memory operations) before it counts itself finished,
    // and the last one reads them with atomic operations.  The frontier and
    // list entries reach the next step through the kernel boundary, so no
    // device-wide fence (a write-back of every L2) is needed here.
    __syncthreads();
    if (threadIdx.x != 0) return;
    __builtin_amdgcn_s_waitcnt(0);
    if (atomicAdd(ctl + S_DONE, 1u) != gridDim.x - 1) return;
    const uint32_t cnt = atomicAdd(ctl + K_CNT, 0u);
    const uint32_t kmin = atomicMin(ctl + K_MIN, 0xffffffffu);
    const uint32_t kept = atomicAdd(ctl + K_KEPT, 0u);
    if (mode == M_SCAN) {
        ctl[S_LIVE] = kept;
        ctl[S_LBUF] ^= 1u;
        ctl[S_FIRST] = 0u;
        if (cnt == 0) {
            if (kmin == 0xffffffffu) ctl[S_MODE] = M_END;   // nothing live
            else ctl[S_LEVEL] = (uint32_t)max(level + 1, (int32_t)kmin);
        } else {
            ctl[S_MAXCORE] = (uint32_t)level;
            ctl[S_MODE] = M_PROCESS;
            ctl[S_CIN] = cnt;
            ctl[S_FBUF] = 0u;
        }
    } else if (cnt == 0) {
        ctl[S_LEVEL] = (uint32_t)(level + 1);
        ctl[S_MODE] = M_SCAN;
    } else {
        ctl[S_CIN] = cnt;
        ctl[S_FBUF] ^= 1u;
    }
    ctl[K_CNT] = 0u;
    ctl[K_MIN] = 0xffffffffu;
    ctl[K_KEPT] = 0u;
    ctl[S_DONE] = 0u;
}

// ------------------------------------------------ h-index fixed point ---
constexpr int32_t kHBins = 4096;      // histogram bins: values capped below this
constexpr int kHWaves = 4;            // waves per workgroup (a histogram each)
constexpr int kMaxRounds = 4096;

// Degree histogram (degrees capped at kHBins), counted per workgroup in LDS
// first: most vertices share a few small degrees, and one global atomic per
// vertex on those few words would queue for milliseconds.
__global__ void __launch_bounds__(kCoreBlock) k_deg_hist(const int32_t *__restrict__ off,
                                                         int32_t n, uint32_t *hist) {
    __shared__ uint32_t local[kHBins + 1];
    for (int32_t b = threadIdx.x; b <= kHBins; b += kCoreBlock) local[b] = 0u;
    __syncthreads();
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&local[min(off[v + 1] - off[v], kHBins)], 1u);
    __syncthreads();
    for (int32_t b = threadIdx.x; b <= kHBins; b += kCoreBlock)
        if (local[b]) atomicAdd(&hist[b], local[b]);
}

// Upper bound of every core number: the largest h with at least h + 1
// vertices of degree >= h (a k-core has k + 1 vertices of degree >= k).
// 0xffffffff when that reaches kHBins.  One workgroup: each thread sums a
// run of bins, a suffix scan over the runs, then each thread finds the
// largest qualifying h in its run.
__global__ void __launch_bounds__(kCoreBlock) k_core_ub(const uint32_t *hist, uint32_t *ctl) {
    __shared__ uint64_t s_part[kCoreWaves];
    __shared__ int32_t s_best[kCoreWaves];
    constexpr int32_t kBins = kHBins + 1;
    constexpr int32_t kPer = (kBins + kCoreBlock - 1) / kCoreBlock;
    const int tid = threadIdx.x, lane = lane_id(), wid = tid / kWave;
    const int32_t b0 = min(kBins, tid * kPer), b1 = min(kBins, b0 + kPer);
    uint64_t own = 0;
    for (int32_t b = b0; b < b1; b++) own += hist[b];
    const uint64_t wscan = wave_incl_scan(own);
    if (lane == kWave - 1) s_part[wid] = wscan;
    __syncthreads();
    uint64_t before = 0, total = 0;
    for (int w = 0; w < kCoreWaves; w++) {
        if (w < wid) before += s_part[w];
        total += s_part[w];
    }
    uint64_t atleast = total - (before + wscan);   // vertices of degree >= b1
    int32_t best = -1;
    for (int32_t b = b1 - 1; b >= b0; b--) {
        atleast += hist[b];
        if (atleast >= (uint64_t)b + 1) {
            best = b;
            break;
        }
    }
    best = wave_max(best);
    if (lane == 0) s_best[wid] = best;
    __syncthreads();
    if (tid == 0) {
        int32_t ub = 0;
        for (int w = 0; w < kCoreWaves; w++) ub = max(ub, s_best[w]);
        ctl[H_UB] = ub >= kHBins ? 0xffffffffu : (uint32_t)ub;
    }
}

__global__ void __launch_bounds__(kCoreBlock) k_hcore_init(const int32_t *__restrict__ off,
                                                           int32_t n, const uint32_t *ctl,
                                                           int32_t *core, uint8_t *act) {
    const int32_t ub = (int32_t)ctl[H_UB];
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        core[v] = min(off[v + 1] - off[v], ub);
        act[v] = 1;
    }
}

constexpr int32_t kBigD = 512;        // vertices of higher degree take a whole workgroup

// One round (see above).  A wave takes 64 consecutive vertices and
// evaluates the active ones of degree <= kBigD among them in turn; those of
// higher degree go to big[] (count bigcnt[round]) for k_hcore_big.
// cnt[round] counts the values that dropped; a round after one without a
// drop does nothing.
__global__ void __launch_bounds__(kCoreBlock) k_hcore_round(const int32_t *__restrict__ off,
                                                            const int32_t *__restrict__ adj,
                                                            int32_t n, int32_t *core,
                                                            uint8_t *act_in, uint8_t *act_out,
                                                            uint32_t *cnt, int32_t *big,
                                                            uint32_t *bigcnt, int32_t round) {
    __shared__ uint32_t s_hist[kHWaves][kBigD + 1];
    if (round > 0 && cnt[round - 1] == 0) return;
    const int lane = lane_id();
    uint32_t *hist = s_hist[threadIdx.x / kWave];
    const int64_t nwaves = (int64_t)gridDim.x * kHWaves;
    uint32_t drops = 0;
    for (int64_t c0 = ((int64_t)blockIdx.x * kHWaves + threadIdx.x / kWave) * kWave; c0 < n;
         c0 += nwaves * kWave) {
        const int64_t mine = c0 + lane;
        const bool a = mine < n && act_in[mine];
        if (a) act_in[mine] = 0;   // consumed; a neighbour's drop may set it again
        uint64_t mask = __ballot(a);
        while (mask) {
            const int32_t v = (int32_t)(c0 + __builtin_ctzll(mask));
            mask &= mask - 1ull;
            const int32_t c = core[v];
            const int32_t s = off[v], d = off[v + 1] - s;
            if (c <= 0) continue;
            if (d > kBigD) {
                if (lane == 0) big[atomicAdd(&bigcnt[round], 1u)] = v;
                continue;
            }
            int32_t h;
            if (d <= kWave) {
                const int32_t x = lane < d ? core[adj[s + lane]] : 0;
                const int32_t k = __popcll(__ballot(x >= c));
                if (k >= c) continue;
                // the largest h in [k, c - 1] with at least h values >= h
                int32_t lo = k, hi = c - 1;
                while (lo < hi) {
                    const int32_t mid = (lo + hi + 1) >> 1;
                    if (__popcll(__ballot(x >= mid)) >= mid) lo = mid;
                    else hi = mid - 1;
                }
                h = lo;
            } else {
                // histogram of min(value, c) over bins 0..c (c <= d <= kBigD);
                // the previous vertex's reads of it come first
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
                for (int32_t b = lane; b <= c; b += kWave) hist[b] = 0u;
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                // four gathers in flight per lane (d <= 512: at most two passes)
                for (int32_t j0 = lane; j0 < d; j0 += 4 * kWave) {
                    int32_t u[4], x[4];
#pragma unroll
                    for (int q = 0; q < 4; q++) {
                        const int32_t j = j0 + q * kWave;
                        u[q] = j < d ? adj[s + j] : -1;
                    }
#pragma unroll
                    for (int q = 0; q < 4; q++) x[q] = u[q] >= 0 ? core[u[q]] : -1;
#pragma unroll
                    for (int q = 0; q < 4; q++)
                        if (x[q] >= 0) atomicAdd(&hist[min(x[q], c)], 1u);
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
                const int32_t k = (int32_t)hist[c];   // values >= c
                if (k >= c) continue;
                // lanes own runs of bins below c; S(b) = values >= b
                const int32_t per = (c + kWave - 1) / kWave;
                const int32_t b0 = min(c, lane * per), b1 = min(c, b0 + per);
                uint32_t own = 0;
                for (int32_t b = b0; b < b1; b++) own += hist[b];
                const uint32_t upto = wave_incl_scan(own);
                const uint32_t total = __shfl(upto, kWave - 1, kWave);
                uint32_t run = (uint32_t)k + (total - upto);   // values >= b1
                int32_t best = -1;
                for (int32_t b = b1 - 1; b >= b0; b--) {
                    run += hist[b];
                    if (run >= (uint32_t)b) {
                        best = b;
                        break;
                    }
                }
                h = wave_max(best);
            }
            if (h >= c) continue;
            if (lane == 0) core[v] = h;
            drops++;
            // neighbours whose value is above h may drop in turn
            for (int32_t j = lane; j < d; j += kWave) {
                const int32_t u = adj[s + j];
                if (core[u] > h) act_out[u] = 1;
            }
        }
    }
    if (lane == 0 && drops) atomicAdd(&cnt[round], drops);
}

// The round's vertices of degree above kBigD, a workgroup each: the same
// evaluation with the workgroup's 256 threads (four gathers in flight each)
// and one histogram in LDS.
__global__ void __launch_bounds__(kCoreBlock) k_hcore_big(const int32_t *__restrict__ off,
                                                          const int32_t *__restrict__ adj,
                                                          int32_t *core, uint8_t *act_out,
                                                          uint32_t *cnt, const int32_t *big,
                                                          const uint32_t *bigcnt, int32_t round) {
    __shared__ uint32_t hist[kHBins];
    __shared__ uint32_t s_part[kCoreWaves];
    __shared__ int32_t s_best[kCoreWaves];
    const int tid = threadIdx.x, lane = lane_id(), wid = tid / kWave;
    const uint32_t nb = bigcnt[round];
    uint32_t drops = 0;
    for (uint32_t i = blockIdx.x; i < nb; i += gridDim.x) {
        const int32_t v = big[i];
        const int32_t c = core[v];   // only this workgroup changes it in this round
        const int32_t s = off[v], d = off[v + 1] - s;
        __syncthreads();   // the previous vertex's reads of hist come first
        for (int32_t b = tid; b <= c; b += kCoreBlock) hist[b] = 0u;
        __syncthreads();
        for (int32_t j0 = tid; j0 < d; j0 += 4 * kCoreBlock) {
            int32_t u[4], x[4];
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int32_t j = j0 + q * kCoreBlock;
                u[q] = j < d ? adj[s + j] : -1;
            }
#pragma unroll
            for (int q = 0; q < 4; q++) x[q] = u[q] >= 0 ? core[u[q]] : -1;
#pragma unroll
            for (int q = 0; q < 4; q++)
                if (x[q] >= 0) atomicAdd(&hist[min(x[q], c)], 1u);
        }
        __syncthreads();
        const int32_t k = (int32_t)hist[c];
        if (k >= c) continue;   // the same for every thread
        // threads own runs of bins below c; a workgroup scan of their sums
        const int32_t per = (c + kCoreBlock - 1) / kCoreBlock;
        const int32_t b0 = min(c, tid * per), b1 = min(c, b0 + per);
        uint32_t own = 0;
        for (int32_t b = b0; b < b1; b++) own += hist[b];
        const uint32_t wscan = wave_incl_scan(own);
        if (lane == kWave - 1) s_part[wid] = wscan;
        __syncthreads();
        uint32_t before = 0, total = 0;
        for (int w = 0; w < kCoreWaves; w++) {
            if (w < wid) before += s_part[w];
            total += s_part[w];
        }
        const uint32_t upto = before + wscan;
        uint32_t run = (uint32_t)k + (total - upto);   // values >= b1
        int32_t best = -1;
        for (int32_t b = b1 - 1; b >= b0; b--) {
            run += hist[b];
            if (run >= (uint32_t)b) {
                best = b;
                break;
            }
        }
        best = wave_max(best);
        if (lane == 0) s_best[wid] = best;
        __syncthreads();
        int32_t h = -1;
        for (int w = 0; w < kCoreWaves; w++) h = max(h, s_best[w]);
        if (h >= c) continue;
        if (tid == 0) {
            core[v] = h;
            drops++;
        }
        for (int32_t j = tid; j < d; j += kCoreBlock) {
            const int32_t u = adj[s + j];
            if (core[u] > h) act_out[u] = 1;
        }
    }
    if (tid == 0 && drops) atomicAdd(&cnt[round], drops);
}

__global__ void __launch_bounds__(kCoreBlock) k_core_max(const int32_t *__restrict__ core,
                                                         int32_t n, uint32_t *ctl) {
    __shared__ int32_t s_mx[kCoreWaves];
    int32_t mx = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        mx = max(mx, core[v]);
    mx = wave_max(mx);
    if (lane_id() == 0) s_mx[threadIdx.x / kWave] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {   // one atomic per workgroup
        for (int w = 1; w < kCoreWaves; w++) mx = max(mx, s_mx[w]);
        if (mx > 0) atomicMax(ctl + H_MAXC, (uint32_t)mx);
    }
}

__device__ __forceinline__ int32_t key_of(const int32_t *__restrict__ off,
                                          const int32_t *__restrict__ core, int32_t v) {
    return core ? core[v] : off[v + 1] - off[v];
}

// Out-degree of every row under the key order (a wave per row).
__global__ void __launch_bounds__(kCoreBlock) k_core_key(const int32_t *__restrict__ off,
                                                         const int32_t *__restrict__ core,
                                                         int32_t n, int32_t S, int32_t *key) {
    const int32_t cap = (int32_t)((1u << S) - 1u);
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        key[v] = (core[v] << S) | min(off[v + 1] - off[v], cap);
}

__global__ void __launch_bounds__(kCoreBlock) k_key_count(const int32_t *__restrict__ off,
                                                          const int32_t *__restrict__ adj,
                                                          int32_t n,
                                                          const int32_t *__restrict__ core,
                                                          int32_t *outcnt) {
    const int lane = lane_id();
    const int64_t nwaves = (int64_t)gridDim.x * kCoreWaves;
    for (int64_t r = (int64_t)blockIdx.x * kCoreWaves + threadIdx.x / kWave; r < n; r += nwaves) {
        const int32_t u = (int32_t)r, ku = key_of(off, core, u), e = off[u + 1];
        int32_t c = 0;
        for (int32_t j = off[u] + lane; j < e; j += kWave) {
            const int32_t v = adj[j];
            c += rank_less(ku, u, key_of(off, core, v), v) ? 1 : 0;
        }
        c = wave_sum(c);
        if (lane == 0) outcnt[u] = c;
    }
}

__global__ void __launch_bounds__(kCoreBlock) k_key_fill(const int32_t *__restrict__ off,
                                                         const int32_t *__restrict__ adj,
                                                         int32_t n,
                                                         const int32_t *__restrict__ core,
                                                         const int32_t *__restrict__ dag_off,
                                                         int32_t *dag_adj, int32_t *dag_src,
                                                         uint32_t *ctl) {
    const int lane = lane_id();
    const int64_t nwaves = (int64_t)gridDim.x * kCoreWaves;
    int32_t maxo = 0;
    for (int64_t r = (int64_t)blockIdx.x * kCoreWaves + threadIdx.x / kWave; r < n; r += nwaves) {
        const int32_t u = (int32_t)r, ku = key_of(off, core, u), e = off[u + 1];
        int32_t base = dag_off[u];
        for (int32_t j0 = off[u]; j0 < e; j0 += kWave) {
            const int32_t j = j0 + lane;
            int32_t v = 0;
            bool keep = false;
            if (j < e) {
                v = adj[j];
                keep = rank_less(ku, u, key_of(off, core, v), v);
            }
            const uint64_t mask = __ballot(keep);
            if (keep) {
                const int32_t p = base + lanes_below(mask);
                dag_adj[p] = v;
                dag_src[p] = u;
            }
            base += __popcll(mask);
        }
        maxo = max(maxo, base - dag_off[u]);
    }
    maxo = wave_max(maxo);
    if (lane == 0 && maxo > 0) atomicMax(ctl + C_MAX_OUT, (uint32_t)maxo);
}

struct CoreWs {
    int32_t *deg, *core, *F, *F2, *L, *L2, *outcnt;
    int64_t *scan_tmp;
    uint32_t *ctl;
    uint32_t *hist, *rounds;   // degree histogram; drops per h-index round
    uint32_t *bigcnt;          // high-degree vertices to evaluate per round (listed in F)
    uint8_t *act0, *act1;      // active flags of the h-index rounds
};

CoreWs core_layout(int32_t n, void *base, uint64_t *bytes) {
    Carve c(base, ~0ull);
    const uint64_t n1 = (uint64_t)n + 1;
    CoreWs W;
    W.deg = c.take<int32_t>(n1);
    W.core = c.take<int32_t>(n1);
    W.F = c.take<int32_t>(n1);
    W.F2 = c.take<int32_t>(n1);
    W.L = c.take<int32_t>(n1);
    W.L2 = c.take<int32_t>(n1);
    W.outcnt = c.take<int32_t>(n1);
    W.scan_tmp = c.take<int64_t>(scan_tmp_words(n1));
    W.ctl = c.take<uint32_t>(C_WORDS);
    W.hist = c.take<uint32_t>(kHBins + 1);
    W.rounds = c.take<uint32_t>(kMaxRounds);
    W.bigcnt = c.take<uint32_t>(kMaxRounds);
    W.act0 = c.take<uint8_t>(n1);
    W.act1 = c.take<uint8_t>(n1);
    if (bytes) *bytes = c.used;
    return W;
}

unsigned vgrid(int64_t items) {
    return (unsigned)std::max<int64_t>(
        1, std::min<int64_t>((items + kCoreBlock - 1) / kCoreBlock, (int64_t)cu_count() * 16));
}

unsigned wgrid(int64_t rows) {
    return (unsigned)std::max<int64_t>(
        1, std::min<int64_t>((rows + kCoreWaves - 1) / kCoreWaves, (int64_t)cu_count() * 16));
}

// A small pinned host buffer for the per-round counters (allocated once per
// process; pageable copies cost several times more per round trip).  It is
// shared by every thread, so read_u32 holds its mutex from the copy to the
// copy-out: concurrent orientations (other graphs, other streams, other
// threads) take turns at the buffer instead of reading each other's words.
std::mutex &pinned_mutex() {
    static std::mutex mu;
    return mu;
}

uint32_t *pinned_words_locked() {
    static uint32_t *p = nullptr;
    if (!p) {
        void *q = nullptr;
        if (hipHostMalloc(&q, sizeof(uint32_t) * C_WORDS, hipHostMallocDefault) == hipSuccess)
            p = static_cast<uint32_t *>(q);
    }
    return p;
}

gpm_status read_u32(const uint32_t *d, uint32_t *h, int count, hipStream_t st) {
    std::lock_guard<std::mutex> lock(pinned_mutex());
    uint32_t *pin = pinned_words_locked();
    GPM_HIP(hipMemcpyAsync(pin ? pin : h, d, sizeof(uint32_t) * count, hipMemcpyDeviceToHost,
                           st));
    GPM_HIP(hipStreamSynchronize(st));
    if (pin)
        for (int i = 0; i < count; i++) h[i] = pin[i];
    return GPM_OK;
}

}  // namespace

uint64_t orient_scratch_bytes(const gpm_graph *g) {
    uint64_t b = 0;
    core_layout(g->n, nullptr, &b);
    return b;
}

// Steps queued per read of the state (RMAT-20 takes about 2,000 steps).
constexpr int kStepsPerTrip = 32;

// Rounds queued per read of the last round's count.
constexpr int kRoundsPerTrip = 8;

// The h-index fixed point; *done = false when the graph is left to the
// peeling (bound above kHBins - 1, or more than kMaxRounds rounds), or with
// GPM_CORE_PEEL=1 in the environment (for comparison).
static gpm_status core_numbers_hindex(const gpm_graph *g, const CoreWs &W, hipStream_t st,
                                      int32_t *max_core, bool *done) {
    *done = false;
    const char *env = getenv("GPM_CORE_PEEL");
    if (env && env[0] == '1') return GPM_OK;
    const int32_t n = g->n;
    GPM_HIP(fill_u32(W.ctl, 0, C_WORDS, st));
    GPM_HIP(fill_u32(W.hist, 0, kHBins + 1, st));
    GPM_HIP(fill_u32(W.rounds, 0, kMaxRounds, st));
    GPM_HIP(fill_u32(W.bigcnt, 0, kMaxRounds, st));
    GPM_HIP(fill_u32(reinterpret_cast<uint32_t *>(W.act1), 0, ((uint64_t)n + 4) / 4, st));
    hipLaunchKernelGGL(k_deg_hist, dim3(vgrid(n)), dim3(kCoreBlock), 0, st, g->off, n, W.hist);
    hipLaunchKernelGGL(k_core_ub, dim3(1), dim3(kCoreBlock), 0, st, W.hist, W.ctl);
    GPM_LAUNCH_CHECK("k_core_ub");
    uint32_t h[C_WORDS];
    gpm_status rc = read_u32(W.ctl, h, C_WORDS, st);
    if (rc) return rc;
    if (h[H_UB] == 0xffffffffu) return GPM_OK;
    Span sp("k_hcore_round", st);
    hipLaunchKernelGGL(k_hcore_init, dim3(vgrid(n)), dim3(kCoreBlock), 0, st, g->off, n, W.ctl,
                       W.core, W.act0);
    GPM_LAUNCH_CHECK("k_hcore_init");
    const unsigned grid = (unsigned)std::max(1, cu_count() * 4);
    for (int32_t r0 = 0; r0 < kMaxRounds; r0 += kRoundsPerTrip) {
        for (int32_t r = r0; r < r0 + kRoundsPerTrip; r++) {
            hipLaunchKernelGGL(k_hcore_round, dim3(grid), dim3(kHWaves * kWave), 0, st, g->off,
                               g->adj, n, W.core, (r & 1) ? W.act1 : W.act0,
                               (r & 1) ? W.act0 : W.act1, W.rounds, W.F, W.bigcnt, r);
            hipLaunchKernelGGL(k_hcore_big, dim3(grid), dim3(kCoreBlock), 0, st, g->off, g->adj,
                               W.core, (r & 1) ? W.act0 : W.act1, W.rounds, W.F, W.bigcnt, r);
        }
        GPM_LAUNCH_CHECK("k_hcore_round");
        uint32_t last = 1;
        rc = read_u32(W.rounds + r0 + kRoundsPerTrip - 1, &last, 1, st);
        if (rc) return rc;
        if (last == 0) {
            hipLaunchKernelGGL(k_core_max, dim3(vgrid(n)), dim3(kCoreBlock), 0, st, W.core, n,
                               W.ctl);
            GPM_LAUNCH_CHECK("k_core_max");
            rc = read_u32(W.ctl, h, C_WORDS, st);
            if (rc) return rc;
            *max_core = (int32_t)h[H_MAXC];
            *done = true;
            return GPM_OK;
        }
    }
    return GPM_OK;   // not settled within kMaxRounds rounds: peel instead
}

static gpm_status core_numbers_run(const gpm_graph *g, const CoreWs &W, hipStream_t st,
                                   int32_t *max_core) {
    bool done = false;
    gpm_status hrc = core_numbers_hindex(g, W, st, max_core, &done);
    if (hrc || done) return hrc;
    const int32_t n = g->n;
    hipLaunchKernelGGL(k_core_init, dim3(vgrid(n)), dim3(kCoreBlock), 0, st, g->off, n, W.deg,
                       W.core);
    GPM_LAUNCH_CHECK("k_core_init");
    GPM_HIP(fill_u32(W.ctl, 0, C_WORDS, st));
    GPM_HIP(fill_u32(W.ctl + K_MIN, 0xffffffffu, 1, st));
    GPM_HIP(fill_u32(W.ctl + S_FIRST, 1u, 1, st));
    // one workgroup per CU: most steps are small and a step's cost is
    // mostly its launch and completion, which grow with the grid (RMAT-20:
    // 17.8 ms at 256 workgroups, 18.1 at 128, 20.4 at 512, 25.3 at 1024)
    const unsigned pgrid = (unsigned)std::max(1, cu_count());
    // a level with removals takes a scan that removes a vertex, sub-rounds
    // that each remove one more but the last, and at most one skipping scan
    // before it; so at most 4n + 1 steps
    const int64_t max_trips = (4 * (int64_t)n + 1) / kStepsPerTrip + 2;
    uint32_t h[C_WORDS];
    Span sp("k_core_step", st);
    for (int64_t trip = 0;; trip++) {
        if (trip > max_trips) return fail(GPM_DEVICE_ERROR, "core peeling did not finish");
        for (int r = 0; r < kStepsPerTrip; r++)
            hipLaunchKernelGGL(k_core_step, dim3(pgrid), dim3(kCoreBlock), 0, st, g->off, g->adj,
                               n, W.deg, W.core, W.F, W.F2, W.L, W.L2, W.ctl);
        GPM_LAUNCH_CHECK("k_core_step");
        gpm_status rc = read_u32(W.ctl, h, C_WORDS, st);
        if (rc) return rc;
        if (h[S_MODE] == M_END) break;
    }
    *max_core = (int32_t)h[S_MAXCORE];
    return GPM_OK;
}

gpm_status graph_orient(gpm_graph *g, int32_t order, void *scratch, uint64_t scratch_bytes,
                        int32_t *d_core, hipStream_t st) {
    uint64_t need = 0;
    CoreWs W = core_layout(g->n, scratch, &need);
    if (need > scratch_bytes) return fail(GPM_OUT_OF_MEMORY, "scratch smaller than required");
    const int32_t n = g->n;
    Span sp(order == GPM_ORIENT_CORE ? "graph_orient_core" : "graph_orient_degree", st);
    GPM_HIP(fill_u32(W.ctl, 0, C_WORDS, st));
    const int32_t *key = nullptr;
    if (order == GPM_ORIENT_CORE || d_core) {
        int32_t max_core = 0;
        gpm_status rc = core_numbers_run(g, W, st, &max_core);
        if (rc) return rc;
        if (d_core)
            GPM_HIP(hipMemcpyAsync(d_core, W.core, sizeof(int32_t) * (size_t)n,
                                   hipMemcpyDeviceToDevice, st));
        if (order == GPM_ORIENT_CORE) {
            int bits = 0;
            while (bits < 31 && (max_core >> bits) != 0) bits++;
            // the local-graph kernels order each root's out-neighbours by the
            // same key, so it is kept with the graph
            hipLaunchKernelGGL(k_core_key, dim3(vgrid(n)), dim3(kCoreBlock), 0, st, g->off,
                               W.core, n, 31 - bits, g->okey);
            GPM_LAUNCH_CHECK("k_core_key");
            key = g->okey;
        }
    }
    hipLaunchKernelGGL(k_key_count, dim3(wgrid(n)), dim3(kCoreBlock), 0, st, g->off, g->adj, n,
                       key, W.outcnt);
    GPM_LAUNCH_CHECK("k_key_count");
    GPM_HIP(exclusive_scan_i32(W.outcnt, g->dag_off, (uint64_t)n, W.scan_tmp, st));
    GPM_HIP(fill_u32(W.ctl + C_MAX_OUT, 0, 1, st));
    hipLaunchKernelGGL(k_key_fill, dim3(wgrid(n)), dim3(kCoreBlock), 0, st, g->off, g->adj, n,
                       key, g->dag_off, g->dag_adj, g->dag_src, W.ctl);
    GPM_LAUNCH_CHECK("k_key_fill");
    if (!key) GPM_HIP(degree_key(g->off, n, g->okey, st));
    uint32_t maxo = 0;
    gpm_status rc = read_u32(W.ctl + C_MAX_OUT, &maxo, 1, st);
    if (rc) return rc;
    g->max_out_degree = (int32_t)maxo;
    return GPM_OK;
}

}  // namespace gpm
