// Internal declarations shared by the library's translation units.
// gfx950 (CDNA4) only: wave64, LDS, HIP streams.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>

#include "../../include/gpm.h"

struct gpm_graph {
    int32_t n;
    int64_t m;
    int32_t max_degree;
    int32_t max_out_degree;
    int32_t n_deg_over_65535;   // vertices of degree above 65535
    int32_t *off;       // [n+1] symmetric CSR offsets
    int32_t *adj;       // [2m]
    int32_t *dag_off;   // [n+1] oriented CSR offsets
    int32_t *dag_adj;   // [m]
    int32_t *dag_src;   // [m] source of each arc
    // [n+1] orientation key: arc u -> v iff (okey[u], u) < (okey[v], v);
    // the degrees after a build, the core-value key after a core orientation
    int32_t *okey;
    // Task granularity of the plain path (gpm_tuning; gpm_graph_autotune
    // picks them per graph): pairs per work chunk and workgroups per CU of
    // the triangle classes (out-degree <= 64, <= 256, <= 1024), one-wave
    // workgroups per CU of the clique kernel for roots of out-degree <= 64,
    // and local triangles per 5-clique task
    int64_t tc_tau[3] = {8192, 16384, 65536};
    int32_t tc_bpc[3] = {32, 8, 4};
    int32_t cw_bpc = 32;
    int64_t lg5_slice = 1 << 20;
};

namespace gpm {

constexpr int kWave = 64;

// ---------------------------------------------------------------- errors --
void set_error(const std::string &msg);
const std::string &last_error();  // per thread
gpm_status fail(gpm_status s, const std::string &msg);
gpm_status hip_fail(hipError_t e, const char *what);

#define GPM_HIP(call)                                                   \
    do {                                                                \
        hipError_t _e = (call);                                         \
        if (_e != hipSuccess) return ::gpm::hip_fail(_e, #call);        \
    } while (0)

#define GPM_LAUNCH_CHECK(what)                                          \
    do {                                                                \
        hipError_t _e = hipGetLastError();                              \
        if (_e != hipSuccess) return ::gpm::hip_fail(_e, what);         \
    } while (0)

// ------------------------------------------------------ workspace carving --
// Bump allocator over a caller-provided device buffer; every piece is
// 256-byte aligned.  With base == nullptr it only measures.
struct Carve {
    char *base;
    uint64_t cap;
    uint64_t used = 0;
    Carve(void *b, uint64_t c) : base(static_cast<char *>(b)), cap(c) {}
    template <class T> T *take(uint64_t count) {
        uint64_t bytes = (count * sizeof(T) + 255) & ~uint64_t(255);
        T *p = base ? reinterpret_cast<T *>(base + used) : nullptr;
        used += bytes;
        return p;
    }
    bool fits() const { return used <= cap; }
};

// ------------------------------------------------------------ primitives --
// Fill n 32-bit words with a value (a kernel, so it may sit in a captured
// graph where memset nodes are avoided).
hipError_t fill_u32(void *p, uint32_t value, uint64_t n, hipStream_t s);
// key[v] = off[v + 1] - off[v] for v < n (the degree order's key).
hipError_t degree_key(const int32_t *off, int32_t n, int32_t *key, hipStream_t s);
// Exclusive scan of n int32 counts into out[0..n] (out[n] = total), using
// tmp (scan_tmp_words(n) int64 words).  in and out may alias.
uint64_t scan_tmp_words(uint64_t n);
hipError_t exclusive_scan_i32(const int32_t *in, int32_t *out, uint64_t n, int64_t *tmp,
                              hipStream_t s);
// Same with 64-bit output offsets.
hipError_t exclusive_scan_i64(const int32_t *in, int64_t *out, uint64_t n, int64_t *tmp,
                              hipStream_t s);
// 64-bit counts in, 64-bit offsets out.
hipError_t exclusive_scan_64(const int64_t *in, int64_t *out, uint64_t n, int64_t *tmp,
                             hipStream_t s);

// Optional kernel timing (off by default): when on, span_begin/span_end
// bracket a launch with HIP events recorded on its stream.
bool timing_on();
// While on, the calling thread records no timing spans (for entry points
// that must not allocate).
void spans_suppress(bool on);
void timing_set(bool on);
int timing_read(const char **names, float *ms, uint64_t *units, int cap);
// Attaches work units (a device uint64, copied when this is called, in
// stream order) to the innermost open span; no-op when timing is off.
void span_units(const unsigned long long *d_units, hipStream_t s);
void span_begin(const char *name, hipStream_t s);
void span_end(hipStream_t s);
struct Span {
    hipStream_t s;
    bool on;
    Span(const char *name, hipStream_t st) : s(st), on(timing_on()) {
        if (on) span_begin(name, s);
    }
    ~Span() {
        if (on) span_end(s);
    }
};

// Number of workgroups a persistent kernel launches: enough resident waves
// to cover every CU several times.
int persistent_blocks(int waves_per_block, int blocks_per_cu);
int cu_count();
// Caps cu_count() for the calling thread (0 = no cap).
void set_cu_limit(int limit);

// ---------------------------------------------------------- device side --
#ifdef __HIPCC__
__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Number of set bits of `mask` below the calling lane.
__device__ __forceinline__ int lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

template <class T> __device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

template <class T> __device__ __forceinline__ T wave_max(T x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        T y = __shfl_xor(x, o, 64);
        x = x > y ? x : y;
    }
    return x;
}

// Inclusive prefix sum across the wave.
template <class T> __device__ __forceinline__ T wave_incl_scan(T x) {
    const int l = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T y = __shfl_up(x, o, 64);
        if (l >= o) x += y;
    }
    return x;
}

// Degree order of Appendix B.2: u precedes v iff deg(u) < deg(v), ties by id.
__device__ __forceinline__ bool rank_less(int32_t du, int32_t u, int32_t dv, int32_t v) {
    return du < dv || (du == dv && u < v);
}

// 128-bit unsigned accumulation into two 64-bit words (lo at p[0], hi at
// p[1]) with carry propagation; concurrent adds commute.
__device__ __forceinline__ void atomic_add_u128(unsigned long long *p, unsigned __int128 x) {
    unsigned long long lo = (unsigned long long)x;
    unsigned long long hi = (unsigned long long)(x >> 64);
    unsigned long long old = atomicAdd(p, lo);
    if (old + lo < old) hi += 1;
    if (hi) atomicAdd(p + 1, hi);
}

// Sum of a 128-bit value over the 64 lanes of a wave (every lane gets it).
__device__ __forceinline__ unsigned __int128 wave_sum_u128(unsigned __int128 x) {
    uint64_t lo = (uint64_t)x, hi = (uint64_t)(x >> 64);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint64_t lo2 = __shfl_xor(lo, o, 64), hi2 = __shfl_xor(hi, o, 64);
        const uint64_t s = lo + lo2;
        hi = hi + hi2 + (s < lo ? 1 : 0);
        lo = s;
    }
    return ((unsigned __int128)hi << 64) | lo;
}

// ------------------------------------------------- LDS membership hash ---
// Open addressing with linear probing over a power-of-two table of int32
// keys (-1 = empty) in LDS, multiplicative hashing.  Used to test whether a
// vertex is one of a root's out-neighbours (and to find its local index)
// with one or two LDS reads instead of a binary search.

// Open addressing with linear probing in LDS; a key's probe sequence starts
// at the first slot of a bucket of 4, so a lookup can read 4 slots at once
// (one 16-byte LDS read) and visits the slots in the order an insert does.
// Key arrays are 16-byte aligned with at least 64 slots.
__device__ __forceinline__ uint32_t lds_hash_slot(int32_t key, int32_t bits) {
    return (((uint32_t)key * 0x9E3779B1u) >> (32 - bits)) & ~3u;
}

// Smallest table size exponent with 2^bits >= f * d (load factor <= 1/f),
// at least 6 (64 slots).  At load 1/8 a 4-slot bucket overflows for about
// 0.2% of lookups, at 1/4 for about 2%: with 128 lookups per step, the
// wave's second probe round is the exception rather than the rule.
__device__ __forceinline__ int32_t lds_hash_bits(int32_t d, int32_t f = 4) {
    int32_t b = 6;
    while ((1 << b) < f * d) b++;
    return b;
}

// Inserts distinct key with value val (vals may be null).
__device__ __forceinline__ void lds_hash_insert(int32_t *keys, int16_t *vals, int32_t bits,
                                                int32_t key, int32_t val) {
    const uint32_t mask = (1u << bits) - 1u;
    uint32_t h = lds_hash_slot(key, bits);
    for (;;) {
        if (atomicCAS(&keys[h], -1, key) == -1) {
            if (vals) vals[h] = (int16_t)val;
            return;
        }
        h = (h + 1) & mask;
    }
}

// Block-wide exclusive scan of PER values per thread (thread t owns entries
// t*PER .. t*PER+PER-1): pre[i+1] = sum of entries 0..i for i < d, pre[0] =
// 0.  s_sum holds NT/64 words of LDS.  Ends with a barrier.
template <int NT, int PER>
__device__ void block_prefix(const int32_t (&val)[PER], int32_t d, int32_t *pre, int32_t *s_sum) {
    const int tid = threadIdx.x, lane = lane_id(), wid = tid / 64;
    int32_t mysum = 0;
#pragma unroll
    for (int q = 0; q < PER; q++) mysum += val[q];
    const int32_t inc = wave_incl_scan(mysum);
    if (NT > 64) {
        if (lane == 63) s_sum[wid] = inc;
        __syncthreads();
    }
    int32_t run = inc - mysum;
    if (NT > 64)
        for (int q = 0; q < wid; q++) run += s_sum[q];
#pragma unroll
    for (int q = 0; q < PER; q++) {
        const int32_t i = tid * PER + q;
        run += val[q];
        if (i < d) pre[i + 1] = run;
    }
    if (tid == 0) pre[0] = 0;
    __syncthreads();
}

// --------------------------------------------- staged roots and pairs ---
// The pairs of a root u of the degree-ordered DAG are (v_j, w) with v_j the
// j-th out-neighbour of u and w in N+(v_j), numbered q = 0 .. W_u - 1 in
// (j, position of w) order.  A staged root holds in LDS
//   pre[j]   first pair number of segment j (pre[d] = W_u),
//   offj[j]  dag_off[v_j] - pre[j], so pair q of segment j is arc offj[j] + q,
//   keys/vals  the membership hash of N+(u) (key v_j, value j).

// Stages root u (d out-neighbours starting at arc s) with NT threads, PER
// out-neighbours per thread (NT * PER >= d).  keys must hold 2^hb slots and
// be cleared to -1 before the call; vals may be null.  The hash value of v_j
// is j, or lidx[j] when lidx is given.  verts (may be null) receives v_j at
// its local index.  Ends with a barrier.
template <int NT, int PER>
__device__ void stage_root(const int32_t *__restrict__ dag_off, const int32_t *__restrict__ dag_adj,
                           int32_t s, int32_t d, int32_t *keys, int16_t *vals, int32_t hb,
                           int32_t *pre, int32_t *offj, int32_t *s_sum,
                           const int16_t *lidx = nullptr, int32_t *verts = nullptr) {
    int32_t dv[PER], vv[PER], st[PER];
#pragma unroll
    for (int k = 0; k < PER; k++) {
        const int32_t i = threadIdx.x * PER + k;
        dv[k] = 0;
        vv[k] = 0;
        st[k] = 0;
        if (i < d) {
            vv[k] = dag_adj[s + i];
            st[k] = dag_off[vv[k]];
            dv[k] = dag_off[vv[k] + 1] - st[k];
        }
    }
    block_prefix<NT, PER>(dv, d, pre, s_sum);
#pragma unroll
    for (int k = 0; k < PER; k++) {
        const int32_t i = threadIdx.x * PER + k;
        if (i < d) {
            offj[i] = st[k] - pre[i];
            const int32_t li = lidx ? (int32_t)lidx[i] : i;
            lds_hash_insert(keys, vals, hb, vv[k], li);
            if (verts) verts[li] = vv[k];
        }
    }
    __syncthreads();
}

// Calls f(j, e_vw, w, slot) for every pair q in [qa, qz) of a staged root
// with d out-neighbours: w is the end of arc e_vw (v = v_j) and slot the
// hash slot of w in keys (2^bits slots), or -1 when w is not an
// out-neighbour of the root.  One pair per lane, U tiles of 64 pairs per
// step, and every round trip to memory is shared by the step's U tiles:
//   - segment: when the step lies inside the current segment j (the usual
//     case: segments are long), its pairs take e = offj[j] + q from two
//     wave-uniform reads; otherwise each lane walks forward from j;
//   - the U loads of w are issued together;
//   - the lookups read a bucket of 4 slots per tile and round, all tiles in
//     the same round, until every lane has a match or an empty slot.
// Wave-uniform qa and qz.
template <int U, class F>
__device__ __forceinline__ void walk_lookup(const int32_t *pre, const int32_t *offj,
                                            const int32_t *__restrict__ dag_adj, int32_t d,
                                            int32_t qa, int32_t qz, const int32_t *keys,
                                            int32_t bits, F &&f) {
    // qa, qz, the segment j and the step bounds live in scalar registers
    qa = __builtin_amdgcn_readfirstlane(qa);
    qz = __builtin_amdgcn_readfirstlane(qz);
    if (qa >= qz) return;
    const int lane = lane_id();
    const uint32_t bmask = (1u << (bits - 2)) - 1u;   // buckets of 4 slots
    const int4 *kb = reinterpret_cast<const int4 *>(keys);
    int32_t lo = 0, hi = d;   // last j with pre[j] <= qa
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (__builtin_amdgcn_readfirstlane(pre[mid]) <= qa) lo = mid; else hi = mid;
    }
    int32_t j = __builtin_amdgcn_readfirstlane(lo);
    for (int32_t qb = qa; qb < qz; qb += U * 64) {
        int32_t jj[U], e[U], w[U], slot[U];
        uint32_t b[U];
        const int32_t seg_end = __builtin_amdgcn_readfirstlane(pre[j + 1]);
        if (qb + U * 64 <= seg_end) {
            // every pair of the step is in segment j (its arcs exist even
            // for lanes past qz)
            const int32_t base = __builtin_amdgcn_readfirstlane(offj[j]) + qb + lane;
#pragma unroll
            for (int t = 0; t < U; t++) {
                jj[t] = j;
                e[t] = base + t * 64;
            }
        } else {
            // lanes past qz take the step's last pair, so every arc exists
            int32_t jc = j;
#pragma unroll
            for (int t = 0; t < U; t++) {
                const int32_t q = min(qb + t * 64 + lane, qz - 1);
                while (pre[jc + 1] <= q) jc++;
                jj[t] = jc;
                e[t] = offj[jc] + q;
            }
        }
        // arc indices are below 2^30, so byte offsets fit 32 bits
        const char *adj_b = reinterpret_cast<const char *>(dag_adj);
#pragma unroll
        for (int t = 0; t < U; t++)
            w[t] = *reinterpret_cast<const int32_t *>(adj_b + ((uint32_t)e[t] << 2));
        bool pend[U];   // lane still looking (lane masks: the logic runs on the scalar unit)
#pragma unroll
        for (int t = 0; t < U; t++) {
            b[t] = lds_hash_slot(w[t], bits) >> 2;
            slot[t] = -1;
            pend[t] = qb + t * 64 + lane < qz;
        }
        // rounds: every lane reads its current bucket (settled lanes re-read
        // theirs) and only pending lanes take the result
        for (;;) {
            int4 kv[U];
#pragma unroll
            for (int t = 0; t < U; t++) kv[t] = kb[b[t]];
            bool more = false;
#pragma unroll
            for (int t = 0; t < U; t++) {
                const int4 k = kv[t];
                const int32_t x = w[t];
                const bool c0 = k.x == x, c1 = k.y == x, c2 = k.z == x, c3 = k.w == x;
                const bool hit = c0 || c1 || c2 || c3;
                const bool empty = (k.x | k.y | k.z | k.w) < 0;
                const int32_t at = (int32_t)(b[t] * 4u) + (c0 ? 0 : (c1 ? 1 : (c2 ? 2 : 3)));
                slot[t] = pend[t] && hit ? at : slot[t];
                pend[t] = pend[t] && !hit && !empty;
                b[t] = (b[t] + 1u) & bmask;
                more = more || pend[t];
            }
            if (!__any(more)) break;
        }
#pragma unroll
        for (int t = 0; t < U; t++)
            if (qb + t * 64 + lane < qz) f(jj[t], e[t], w[t], slot[t]);
        j = __builtin_amdgcn_readlane(jj[U - 1], 63);
    }
}

// Count-only form of walk_lookup: the number of pairs q in [qa, qz) whose
// end w is an out-neighbour of the root, wave-uniform.  No slot is needed,
// so each round's hits are a lane mask (compare results are lane masks
// already) counted on the scalar unit, and the lanes still looking are a
// mask too: about a third of walk_lookup's vector instructions per tile.
template <int U>
__device__ __forceinline__ uint64_t walk_count(const int32_t *pre, const int32_t *offj,
                                               const int32_t *__restrict__ dag_adj, int32_t d,
                                               int32_t qa, int32_t qz, const int32_t *keys,
                                               int32_t bits) {
    qa = __builtin_amdgcn_readfirstlane(qa);
    qz = __builtin_amdgcn_readfirstlane(qz);
    uint64_t total = 0;
    if (qa >= qz) return 0;
    const int lane = lane_id();
    const uint32_t bmask = (1u << (bits - 2)) - 1u;
    const int4 *kb = reinterpret_cast<const int4 *>(keys);
    int32_t lo = 0, hi = d;
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (__builtin_amdgcn_readfirstlane(pre[mid]) <= qa) lo = mid; else hi = mid;
    }
    int32_t j = __builtin_amdgcn_readfirstlane(lo);
    const char *adj_b = reinterpret_cast<const char *>(dag_adj);
    for (int32_t qb = qa; qb < qz; qb += U * 64) {
        int32_t jl = j, e[U], w[U];
        uint32_t b[U];
        uint64_t pend[U];
        const int32_t seg_end = __builtin_amdgcn_readfirstlane(pre[j + 1]);
        if (qb + U * 64 <= seg_end) {
            const int32_t base = __builtin_amdgcn_readfirstlane(offj[j]) + qb + lane;
#pragma unroll
            for (int t = 0; t < U; t++) e[t] = base + t * 64;
        } else {
            int32_t jc = j;
#pragma unroll
            for (int t = 0; t < U; t++) {
                const int32_t q = min(qb + t * 64 + lane, qz - 1);
                while (pre[jc + 1] <= q) jc++;
                e[t] = offj[jc] + q;
            }
            jl = jc;
        }
#pragma unroll
        for (int t = 0; t < U; t++) {
            w[t] = *reinterpret_cast<const int32_t *>(adj_b + ((uint32_t)e[t] << 2));
            pend[t] = __ballot(qb + t * 64 + lane < qz);
        }
#pragma unroll
        for (int t = 0; t < U; t++) b[t] = lds_hash_slot(w[t], bits) >> 2;
        for (;;) {
            int4 kv[U];
#pragma unroll
            for (int t = 0; t < U; t++) kv[t] = kb[b[t]];
            uint64_t more = 0;
#pragma unroll
            for (int t = 0; t < U; t++) {
                const int4 k = kv[t];
                const int32_t x = w[t];
                // one lane mask per compare, combined on the scalar unit
                const uint64_t hit = __ballot(k.x == x) | __ballot(k.y == x) |
                                     __ballot(k.z == x) | __ballot(k.w == x);
                const uint64_t empty = __ballot((k.x | k.y | k.z | k.w) < 0);
                total += (uint64_t)__popcll(hit & pend[t]);
                pend[t] &= ~(hit | empty);
                b[t] = (b[t] + 1u) & bmask;
                more |= pend[t];
            }
            if (!more) break;
        }
        j = __builtin_amdgcn_readlane(jl, 63);
    }
    return total;
}

// splitmix64 finaliser, for the listing checksum.
__device__ __forceinline__ uint64_t fmix64(uint64_t z) {
    z ^= z >> 30; z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27; z *= 0x94D049BB133111EBull;
    z ^= z >> 31;
    return z;
}

// ---------------------------------------------------------- listing ---
// Listing output: a slot counter hands out rows of the caller's buffer while
// it has room (once a wave has seen the counter pass the capacity it stops
// asking); the total and the checksum are kept per lane and added once per
// wave at the end (row_emitter_flush), the written count by the host-side
// finish (min(counter, cap)).
struct RowEmitter {
    unsigned long long *slot_ctr;
    int32_t *buf;
    uint64_t cap;
    uint64_t cached;   // last counter value this lane's wave saw
    uint64_t count;    // per lane
    uint64_t hsum;     // per lane
};

// Checksum term of an embedding: its key sorted ascending, then
// h = L, h = fmix64((h XOR key_i) + 0x9E3779B97F4A7C15) over the key.
template <int L>
__device__ __forceinline__ uint64_t sorted_key_hash(uint64_t (&k)[L]) {
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

// Emits the vertex-induced embedding v (L vertex ids, written in this order)
// for every calling lane; may be called from divergent code (the lowest
// active lane takes the slots for the others).
template <int L>
__device__ __forceinline__ void emit_vertices(RowEmitter &em, const int32_t (&v)[L]) {
    uint64_t key[L];
#pragma unroll
    for (int i = 0; i < L; i++) key[i] = (uint64_t)(uint32_t)v[i];
    em.hsum += sorted_key_hash<L>(key);
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
        int32_t *o = em.buf + slot * (uint64_t)L;
#pragma unroll
        for (int i = 0; i < L; i++) o[i] = v[i];
    }
}

// Adds the wave's totals to result[0] (embeddings) and result[2] (checksum);
// the whole wave must call it.
__device__ __forceinline__ void row_emitter_flush(const RowEmitter &em, unsigned long long *result) {
    const uint64_t c = wave_sum(em.count), h = wave_sum(em.hsum);
    if (lane_id() == 0) {
        if (c) atomicAdd(&result[0], (unsigned long long)c);
        if (h) atomicAdd(&result[2], (unsigned long long)h);
    }
}
#endif

}  // namespace gpm
