// Error reporting, fills, exclusive scans and launch sizing.
#include "gpm_internal.h"

#include <mutex>
#include <vector>

namespace gpm {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

const std::string &last_error() { return g_last_error; }

gpm_status fail(gpm_status s, const std::string &msg) {
    g_last_error = msg;
    return s;
}

gpm_status hip_fail(hipError_t e, const char *what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return GPM_DEVICE_ERROR;
}

// ------------------------------------------------------------------ fill --
__global__ void k_fill_u32(uint32_t *p, uint32_t value, uint64_t n) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = value;
}

hipError_t fill_u32(void *p, uint32_t value, uint64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s,
                       static_cast<uint32_t *>(p), value, n);
    return hipGetLastError();
}

// ------------------------------------------------------------------ scan --
// Three phases over tiles of kTile = 256 threads x 16 items: per-tile sums,
// one workgroup scanning the tile sums, then per-tile local scans plus the
// tile's offset.
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kTile = kScanThreads * kScanItems;

uint64_t scan_tmp_words(uint64_t n) { return (n + kTile - 1) / kTile + 1; }

// Block-wide exclusive scan of one int64 per thread; returns the block total.
__device__ int64_t block_excl_scan(int64_t x, int64_t *sh /*[kScanThreads/64]*/,
                                   int64_t &total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int64_t inc = wave_incl_scan(x);
    if (lane == 63) sh[wid] = inc;
    __syncthreads();
    int64_t base = 0, tot = 0;
    for (int w = 0; w < kScanThreads / 64; w++) {
        if (w < wid) base += sh[w];
        tot += sh[w];
    }
    __syncthreads();
    total = tot;
    return base + inc - x;
}

template <class InT>
__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(const InT *in, uint64_t n,
                                                             int64_t *tile_sums) {
    __shared__ int64_t sh[kScanThreads / 64];
    uint64_t base = (uint64_t)blockIdx.x * kTile;
    int64_t s = 0;
    for (int i = 0; i < kScanItems; i++) {
        uint64_t idx = base + (uint64_t)i * kScanThreads + threadIdx.x;
        if (idx < n) s += in[idx];
    }
    int64_t tot;
    block_excl_scan(s, sh, tot);
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = tot;
}

// One workgroup: exclusive scan of the tile sums in place; total -> tile_sums[ntiles].
__global__ void __launch_bounds__(kScanThreads) k_scan_tiles(int64_t *tile_sums, uint64_t ntiles) {
    __shared__ int64_t sh[kScanThreads / 64];
    int64_t carry = 0;
    for (uint64_t b = 0; b < ntiles; b += kScanThreads) {
        uint64_t idx = b + threadIdx.x;
        int64_t x = idx < ntiles ? tile_sums[idx] : 0;
        int64_t tot;
        int64_t ex = block_excl_scan(x, sh, tot);
        if (idx < ntiles) tile_sums[idx] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) tile_sums[ntiles] = carry;
}

template <class InT, class OutT>
__global__ void __launch_bounds__(kScanThreads) k_scan_down(const InT *in, OutT *out,
                                                           uint64_t n, const int64_t *tile_sums,
                                                           uint64_t ntiles) {
    __shared__ InT tile[kTile];
    __shared__ int64_t sh[kScanThreads / 64];
    uint64_t base = (uint64_t)blockIdx.x * kTile;
    for (int i = 0; i < kScanItems; i++) {
        int j = i * kScanThreads + threadIdx.x;
        tile[j] = (base + j < n) ? in[base + j] : 0;
    }
    __syncthreads();
    InT v[kScanItems];
    int64_t s = 0;
    for (int i = 0; i < kScanItems; i++) {
        v[i] = tile[threadIdx.x * kScanItems + i];
        s += v[i];
    }
    int64_t tot;
    int64_t run = tile_sums[blockIdx.x] + block_excl_scan(s, sh, tot);
    for (int i = 0; i < kScanItems; i++) {
        uint64_t idx = base + (uint64_t)threadIdx.x * kScanItems + i;
        if (idx < n) out[idx] = (OutT)run;
        run += v[i];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = (OutT)tile_sums[ntiles];
}

template <class InT, class OutT>
static hipError_t scan_impl(const InT *in, OutT *out, uint64_t n, int64_t *tmp, hipStream_t s) {
    uint64_t ntiles = (n + kTile - 1) / kTile;
    if (ntiles == 0) {
        // n == 0: out[0] = 0
        hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kScanThreads), 0, s, tmp, (uint64_t)0);
        hipLaunchKernelGGL((k_scan_down<InT, OutT>), dim3(1), dim3(kScanThreads), 0, s, in, out,
                           (uint64_t)0, (const int64_t *)tmp, (uint64_t)0);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((k_scan_reduce<InT>), dim3((unsigned)ntiles), dim3(kScanThreads), 0, s, in,
                       n, tmp);
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kScanThreads), 0, s, tmp, ntiles);
    hipLaunchKernelGGL((k_scan_down<InT, OutT>), dim3((unsigned)ntiles), dim3(kScanThreads), 0, s,
                       in, out, n, (const int64_t *)tmp, ntiles);
    return hipGetLastError();
}

hipError_t exclusive_scan_i32(const int32_t *in, int32_t *out, uint64_t n, int64_t *tmp,
                              hipStream_t s) {
    return scan_impl<int32_t, int32_t>(in, out, n, tmp, s);
}

hipError_t exclusive_scan_i64(const int32_t *in, int64_t *out, uint64_t n, int64_t *tmp,
                              hipStream_t s) {
    return scan_impl<int32_t, int64_t>(in, out, n, tmp, s);
}

hipError_t exclusive_scan_64(const int64_t *in, int64_t *out, uint64_t n, int64_t *tmp,
                             hipStream_t s) {
    return scan_impl<int64_t, int64_t>(in, out, n, tmp, s);
}

// ---------------------------------------------------------------- timing --
namespace {
struct Rec {
    std::string name;
    hipEvent_t a, b;
    int unit_slot;   // pinned slot holding the span's work units, or -1
};
std::mutex g_tmu;
bool g_timing = false;
std::vector<Rec> g_recs;
std::vector<size_t> g_open;
constexpr int kUnitSlots = 4096;
unsigned long long *g_units = nullptr;   // pinned host slots
int g_units_used = 0;
}  // namespace

// Set while an entry point that must not allocate runs on this thread: its
// kernels record no spans (a span creates events and, for work units, a
// pinned host buffer).
static thread_local bool tls_no_spans = false;

void spans_suppress(bool on) { tls_no_spans = on; }

void span_units(const unsigned long long *d_units, hipStream_t s) {
    if (tls_no_spans) return;
    std::lock_guard<std::mutex> lock(g_tmu);
    if (!g_timing || g_open.empty()) return;
    if (!g_units) {
        void *p = nullptr;
        if (hipHostMalloc(&p, sizeof(unsigned long long) * kUnitSlots, hipHostMallocDefault) !=
            hipSuccess)
            return;
        g_units = static_cast<unsigned long long *>(p);
    }
    if (g_units_used >= kUnitSlots) return;
    const int slot = g_units_used++;
    g_recs[g_open.back()].unit_slot = slot;
    (void)hipMemcpyAsync(g_units + slot, d_units, sizeof(unsigned long long),
                         hipMemcpyDeviceToHost, s);
}

bool timing_on() { return g_timing && !tls_no_spans; }

void span_begin(const char *name, hipStream_t s) {
    std::lock_guard<std::mutex> lock(g_tmu);
    Rec r{name, nullptr, nullptr, -1};
    // timing is best effort: a span whose events cannot be made or recorded
    // keeps its place (so nesting stays paired) and reads back as no time
    if (hipEventCreate(&r.a) != hipSuccess) r.a = nullptr;
    if (hipEventCreate(&r.b) != hipSuccess) r.b = nullptr;
    if (r.a && r.b && hipEventRecord(r.a, s) != hipSuccess) {
        (void)hipEventDestroy(r.a);
        r.a = nullptr;
    }
    g_open.push_back(g_recs.size());
    g_recs.push_back(r);
}

void span_end(hipStream_t s) {
    std::lock_guard<std::mutex> lock(g_tmu);
    if (g_open.empty()) return;
    size_t i = g_open.back();
    g_open.pop_back();
    if (g_recs[i].a && g_recs[i].b && hipEventRecord(g_recs[i].b, s) != hipSuccess) {
        (void)hipEventDestroy(g_recs[i].a);
        g_recs[i].a = nullptr;
    }
}

void timing_set(bool on) {
    std::lock_guard<std::mutex> lock(g_tmu);
    g_timing = on;
}

int timing_read(const char **names, float *ms, uint64_t *units, int cap) {
    std::lock_guard<std::mutex> lock(g_tmu);
    static std::vector<std::string> keep;
    keep.clear();
    int k = 0;
    for (auto &r : g_recs) {
        float t = -1.f;
        if (r.a && r.b && hipEventSynchronize(r.b) == hipSuccess &&
            hipEventElapsedTime(&t, r.a, r.b) != hipSuccess)
            t = -1.f;
        if (k < cap) {
            keep.push_back(r.name);
            if (ms) ms[k] = t;
            if (units) units[k] = r.unit_slot >= 0 ? g_units[r.unit_slot] : 0;
        }
        k++;
        if (r.a) (void)hipEventDestroy(r.a);
        if (r.b) (void)hipEventDestroy(r.b);
    }
    if (names)
        for (int i = 0; i < (int)keep.size(); i++) names[i] = keep[i].c_str();
    g_recs.clear();
    g_open.clear();
    g_units_used = 0;
    return k;
}

// ---------------------------------------------------------- launch sizing --
// Persistent grids are sized from the compute-unit count; a thread may cap
// the count it sees (the serving scheduler does, so that one request's
// persistent kernels leave room for others').
static thread_local int tls_cu_limit = 0;

void set_cu_limit(int limit) { tls_cu_limit = limit > 0 ? limit : 0; }

int cu_count() {
    static int cached = 0;
    static std::mutex mu;
    int c;
    {
        std::lock_guard<std::mutex> lock(mu);
        if (cached == 0) {
            int dev = 0, cus = 0;
            if (hipGetDevice(&dev) == hipSuccess &&
                hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) ==
                    hipSuccess &&
                cus > 0)
                cached = cus;
            else
                cached = 256;
        }
        c = cached;
    }
    return tls_cu_limit > 0 && tls_cu_limit < c ? tls_cu_limit : c;
}

int persistent_blocks(int waves_per_block, int blocks_per_cu) {
    (void)waves_per_block;
    return cu_count() * blocks_per_cu;
}

}  // namespace gpm
