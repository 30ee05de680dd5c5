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
    int32_t *off;       // [n+1] symmetric CSR offsets
    int32_t *adj;       // [2m]
    int32_t *dag_off;   // [n+1] oriented CSR offsets
    int32_t *dag_adj;   // [m]
    int32_t *dag_src;   // [m] source of each arc
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

// splitmix64 finaliser, for the listing checksum.
__device__ __forceinline__ uint64_t fmix64(uint64_t z) {
    z ^= z >> 30; z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27; z *= 0x94D049BB133111EBull;
    z ^= z >> 31;
    return z;
}
#endif

}  // namespace gpm
