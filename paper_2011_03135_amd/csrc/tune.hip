// Per-graph tuning of the plain path's task granularity (Section 4.1 splits
// the work into tasks and leaves their size open).  The knobs: pairs per
// work chunk and workgroups per CU of the three triangle classes, the grid
// of the wave-per-root clique kernel, and local triangles per 5-clique
// task.  The tuner times the calls they govern on
// the graph itself (HIP events on the caller's stream, the median of three
// runs after a warm-up) and walks the knobs one at a time (coordinate
// descent), keeping a change only when it is at least 3% faster.  Counts
// never depend on the tuning.
#include "gpm_internal.h"

#include <algorithm>
#include <vector>

namespace gpm {

gpm_status clique_workspace_bytes(const gpm_graph *g, int32_t k, bool list, uint64_t *bytes);
gpm_status clique_run(const gpm_graph *g, int32_t k, bool list, void *ws, uint64_t ws_bytes,
                      unsigned long long *d_count, int32_t *d_buf, uint64_t cap,
                      unsigned long long *d_result, hipStream_t st);

namespace {

constexpr int64_t kTauLo = 2048, kTauHi = int64_t(1) << 24;
constexpr int32_t kBpcLo = 1, kBpcHi = 64;
constexpr int32_t kCwLo = 8, kCwHi = 1024;
constexpr int64_t kSliceLo = int64_t(1) << 14, kSliceHi = int64_t(1) << 28;
constexpr int32_t kSliceRootMin = 257;   // roots above this out-degree take 5-clique slices
constexpr uint64_t kResultBytes = 256;

void put(gpm_graph *g, const gpm_tuning &t) {
    for (int c = 0; c < 3; c++) {
        g->tc_tau[c] = t.tc_tau[c];
        g->tc_bpc[c] = t.tc_blocks_per_cu[c];
    }
    g->cw_bpc = t.clique_wave_blocks_per_cu;
    g->lg5_slice = t.lg5_slice;
}

}  // namespace

void tuning_get(const gpm_graph *g, gpm_tuning *t) {
    for (int c = 0; c < 3; c++) {
        t->tc_tau[c] = g->tc_tau[c];
        t->tc_blocks_per_cu[c] = g->tc_bpc[c];
    }
    t->clique_wave_blocks_per_cu = g->cw_bpc;
    t->lg5_slice = g->lg5_slice;
}

gpm_status tuning_set(gpm_graph *g, const gpm_tuning *t) {
    for (int c = 0; c < 3; c++) {
        if (t->tc_tau[c] < kTauLo || t->tc_tau[c] > kTauHi)
            return fail(GPM_INVALID_ARGUMENT, "tc_tau outside [2048, 2^24]");
        if (t->tc_blocks_per_cu[c] < kBpcLo || t->tc_blocks_per_cu[c] > kBpcHi)
            return fail(GPM_INVALID_ARGUMENT, "tc_blocks_per_cu outside [1, 64]");
    }
    if (t->clique_wave_blocks_per_cu < kCwLo || t->clique_wave_blocks_per_cu > kCwHi)
        return fail(GPM_INVALID_ARGUMENT, "clique_wave_blocks_per_cu outside [8, 1024]");
    if (t->lg5_slice < kSliceLo || t->lg5_slice > kSliceHi)
        return fail(GPM_INVALID_ARGUMENT, "lg5_slice outside [2^14, 2^28]");
    put(g, *t);
    return GPM_OK;
}

// Workspace of the tuner: a result slot, then a clique workspace for k = 3
// to 5 at the smallest chunk size it tries.
gpm_status autotune_bytes(const gpm_graph *g, uint64_t *bytes) {
    gpm_graph tmp = *g;
    for (int c = 0; c < 3; c++) tmp.tc_tau[c] = kTauLo;
    uint64_t most = 0;
    for (int32_t k = 3; k <= 5; k++) {
        uint64_t b = 0;
        gpm_status rc = clique_workspace_bytes(&tmp, k, false, &b);
        if (rc) return rc;
        most = std::max(most, b);
    }
    *bytes = kResultBytes + most;
    return GPM_OK;
}

gpm_status graph_autotune(gpm_graph *g, void *ws, uint64_t ws_bytes, hipStream_t st,
                          gpm_tuning *chosen) {
    uint64_t need = 0;
    gpm_status rc = autotune_bytes(g, &need);
    if (rc) return rc;
    if (ws_bytes < need) return fail(GPM_OUT_OF_MEMORY, "workspace smaller than required");
    auto *d_res = static_cast<unsigned long long *>(ws);
    void *cws = static_cast<char *>(ws) + kResultBytes;
    const uint64_t cbytes = ws_bytes - kResultBytes;
    hipEvent_t a = nullptr, b = nullptr;
    GPM_HIP(hipEventCreate(&a));
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return fail(GPM_DEVICE_ERROR, "hipEventCreate failed");
    }
    gpm_tuning cur, orig;
    tuning_get(g, &cur);
    orig = cur;
    gpm_status err = GPM_OK;
    // median of three timed calls after one warm-up; a failure ends the tuning
    auto timed = [&](int k) -> float {
        if (err) return 0.f;
        std::vector<float> ms;
        for (int r = 0; r < 4 && !err; r++) {
            hipError_t e = hipEventRecord(a, st);
            if (e == hipSuccess) {
                err = clique_run(g, k, false, cws, cbytes, d_res, nullptr, 0, nullptr, st);
                if (!err) e = hipEventRecord(b, st);
            }
            if (e == hipSuccess && !err) e = hipEventSynchronize(b);
            float x = 0.f;
            if (e == hipSuccess && !err) e = hipEventElapsedTime(&x, a, b);
            if (e != hipSuccess && !err) err = hip_fail(e, "timing a tuning candidate");
            if (r > 0) ms.push_back(x);
        }
        if (err) return 0.f;
        std::sort(ms.begin(), ms.end());
        return ms[ms.size() / 2];
    };
    // tries t as the current tuning; keeps it when 3% faster than best
    auto attempt = [&](const gpm_tuning &t, int k, float &best) {
        put(g, t);
        const float x = timed(k);
        if (!err && x < 0.97f * best) {
            best = x;
            cur = t;
        } else {
            put(g, cur);
        }
    };
    float best3 = timed(3);
    for (int pass = 0; pass < 2 && !err; pass++)
        for (int c = 0; c < 3 && !err; c++) {
            for (const double f : {4.0, 2.0, 0.5, 0.25}) {
                gpm_tuning t = cur;
                t.tc_tau[c] = std::min(kTauHi, std::max(kTauLo, (int64_t)(cur.tc_tau[c] * f)));
                if (t.tc_tau[c] != cur.tc_tau[c]) attempt(t, 3, best3);
            }
            for (const double f : {2.0, 0.5}) {
                gpm_tuning t = cur;
                t.tc_blocks_per_cu[c] = std::min(
                    kBpcHi, std::max(kBpcLo, (int32_t)(cur.tc_blocks_per_cu[c] * f)));
                if (t.tc_blocks_per_cu[c] != cur.tc_blocks_per_cu[c]) attempt(t, 3, best3);
            }
        }
    if (!err) {
        float best4 = timed(4);
        for (const double f : {4.0, 2.0, 0.5}) {
            if (err) break;
            gpm_tuning t = cur;
            t.clique_wave_blocks_per_cu = std::min(
                kCwHi, std::max(kCwLo, (int32_t)(cur.clique_wave_blocks_per_cu * f)));
            if (t.clique_wave_blocks_per_cu != cur.clique_wave_blocks_per_cu) attempt(t, 4, best4);
        }
    }
    if (!err && g->max_out_degree >= kSliceRootMin) {
        float best5 = timed(5);
        for (const double f : {4.0, 2.0, 0.5, 0.25}) {
            if (err) break;
            gpm_tuning t = cur;
            t.lg5_slice = std::min(kSliceHi, std::max(kSliceLo, (int64_t)(cur.lg5_slice * f)));
            if (t.lg5_slice != cur.lg5_slice) attempt(t, 5, best5);
        }
    }
    put(g, err ? orig : cur);   // a failed tuning leaves the handle as it was
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (err) return err;
    if (chosen) *chosen = cur;
    return GPM_OK;
}

}  // namespace gpm
