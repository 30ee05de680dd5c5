// Induced 3- and 4-motif counting by local counting (Section 5: the wedge
// equation and the diamond count from per-edge triangle counts; Appendix A:
// the 3-motif and 4-motif local-counting listings, whose elided final step is
// completed here with per-edge identities).
//
// 3-motifs: wedges (open) = sum_v C(d_v, 2) - 3T, triangles = T.
//
// 4-motifs.  For every undirected edge e = (u, v) with T_e triangles,
// S_u = d_u - T_e - 1 and S_v = d_v - T_e - 1 (the local wedge terms of the
// wedge equation), these sums over edges, each edge visited once, equal
// induced counts (I_*):
//   sum C(T_e, 2)                  = I_diamond + 6 I_K4
//   sum T_e (S_u + S_v)            = 2 I_paw + 4 I_diamond
//   sum S_u S_v                    = I_P4 + 4 I_C4
//   sum C(S_u, 2) + C(S_v, 2)      = 3 I_claw + I_paw
// With I_K4 from 4-clique counting and the number of 4-cycles N_C4 (not
// necessarily induced; N_C4 = I_C4 + I_diamond + 3 I_K4) the system solves
// exactly; every division is checked.
//
// N_C4 comes from the 4-cycle counter (c4.hip).
#include "gpm_internal.h"

#include <algorithm>
#include <climits>

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

namespace {

typedef unsigned __int128 u128;

constexpr int kBlock = 256;

__global__ void k_degrees(const int32_t *off, int32_t n, int32_t *deg) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) deg[i] = off[i + 1] - off[i];
}

// sum_v C(d_v, 2) as 128 bits.
__global__ void __launch_bounds__(kBlock) k_wedge_sum(const int32_t *deg, int32_t n,
                                                      unsigned long long *out) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * kBlock;
    u128 s = 0;
    for (; i < n; i += stride) {
        uint64_t d = (uint64_t)deg[i];
        s += (u128)(d * (d - (d > 0)) / 2);
    }
    s = wave_sum_u128(s);
    if (lane_id() == 0 && s) atomic_add_u128(out, s);
}

// The four per-edge local-count sums, each 128 bits: out[0..7].
__global__ void __launch_bounds__(kBlock) k_lc_sums(const int32_t *__restrict__ dag_src,
                                                    const int32_t *__restrict__ dag_adj,
                                                    const uint32_t *__restrict__ te,
                                                    const int32_t *__restrict__ deg, int64_t m,
                                                    unsigned long long *out) {
    int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * kBlock;
    u128 s1 = 0, s2 = 0, s3 = 0, s4 = 0;
    for (; e < m; e += stride) {
        const uint64_t t = te[e];
        const uint64_t du = (uint64_t)deg[dag_src[e]], dv = (uint64_t)deg[dag_adj[e]];
        const uint64_t su = du - t - 1, sv = dv - t - 1;
        s1 += (u128)(t * (t - (t > 0)) / 2);
        s2 += (u128)t * (su + sv);
        s3 += (u128)su * sv;
        s4 += (u128)(su * (su - (su > 0)) / 2) + (u128)(sv * (sv - (sv > 0)) / 2);
    }
    s1 = wave_sum_u128(s1);
    s2 = wave_sum_u128(s2);
    s3 = wave_sum_u128(s3);
    s4 = wave_sum_u128(s4);
    if (lane_id() == 0) {
        if (s1) atomic_add_u128(out + 0, s1);
        if (s2) atomic_add_u128(out + 2, s2);
        if (s3) atomic_add_u128(out + 4, s3);
        if (s4) atomic_add_u128(out + 6, s4);
    }
}

// ------------------------------------------------------------- combine ---

struct Sums {
    unsigned long long tri;        // T (triangles)
    unsigned long long k4;         // 4-cliques
    unsigned long long lc[8];      // four 128-bit local-count sums
    unsigned long long wedge[2];   // sum_v C(d_v, 2)
    unsigned long long c4[2];      // N_C4
};

__device__ __forceinline__ u128 get128(const unsigned long long *p) {
    return ((u128)p[1] << 64) | p[0];
}

__global__ void k_combine(const Sums *S, int32_t k, unsigned long long *out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const u128 lim = (u128)1 << 64;
    unsigned long long bad = 0;
    if (k == 3) {
        const u128 w = get128(S->wedge), t3 = (u128)3 * S->tri;
        if (w < t3) bad |= 1;
        const u128 wo = w - t3;
        if (wo >= lim) bad |= 2;
        out[0] = (unsigned long long)wo;
        out[1] = S->tri;
        out[2] = bad;
        return;
    }
    const u128 k4 = S->k4;
    const u128 s1 = get128(S->lc + 0), s2 = get128(S->lc + 2), s3 = get128(S->lc + 4),
               s4 = get128(S->lc + 6), nc4 = get128(S->c4);
    u128 dia = 0, paw = 0, c4 = 0, p4 = 0, claw = 0;
    if (s1 < 6 * k4) bad |= 1; else dia = s1 - 6 * k4;
    if (s2 < 4 * dia || ((s2 - 4 * dia) & 1)) bad |= 2; else paw = (s2 - 4 * dia) / 2;
    if (nc4 < dia + 3 * k4) bad |= 4; else c4 = nc4 - dia - 3 * k4;
    if (s3 < 4 * c4) bad |= 8; else p4 = s3 - 4 * c4;
    if (s4 < paw || (s4 - paw) % 3) bad |= 16; else claw = (s4 - paw) / 3;
    const u128 r[6] = {claw, p4, c4, paw, dia, k4};
    for (int i = 0; i < 6; i++) {
        if (r[i] >= lim) bad |= 32;
        out[i] = (unsigned long long)r[i];
    }
    out[6] = bad;
}

struct MotifWs {
    Sums *sums;
    uint32_t *te;
    int32_t *deg;
    uint32_t *ctl;
    void *shared;      // clique workspace (k = 3 or 4), reused in sequence
    void *c4ws;        // 4-cycle counting workspace
    uint64_t shared_bytes, c4_bytes, bytes;
};

MotifWs motif_layout(const gpm_graph *g, int32_t k, void *base) {
    MotifWs W{};
    Carve c(base, ~0ull);
    const uint64_t n1 = (uint64_t)g->n + 1;
    W.sums = c.take<Sums>(1);
    W.ctl = c.take<uint32_t>(16);
    W.deg = c.take<int32_t>(n1);
    if (k == 4) {
        W.te = c.take<uint32_t>((uint64_t)std::max<int64_t>(g->m, 1));
        c4_workspace_bytes(g, false, &W.c4_bytes);
        W.c4ws = c.take<char>(W.c4_bytes);
    }
    uint64_t b3 = 0, b4 = 0;
    clique_workspace_bytes(g, 3, false, &b3);
    if (k == 4) clique_workspace_bytes(g, 4, false, &b4);
    W.shared_bytes = std::max(b3, b4);
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

gpm_status motif_workspace_bytes(const gpm_graph *g, int32_t k, uint64_t *bytes) {
    *bytes = motif_layout(g, k, nullptr).bytes;
    return GPM_OK;
}

gpm_status motif_run(const gpm_graph *g, int32_t k, void *ws, uint64_t ws_bytes,
                     unsigned long long *d_counts, hipStream_t st) {
    MotifWs W = motif_layout(g, k, ws);
    if (W.bytes > ws_bytes) return fail(GPM_OUT_OF_MEMORY, "workspace smaller than required");
    const int32_t n = g->n;
    GPM_HIP(fill_u32(W.sums, 0, sizeof(Sums) / 4, st));
    GPM_HIP(fill_u32(W.ctl, 0, 16, st));
    hipLaunchKernelGGL(k_degrees, dim3(grid_for(n, 256, 8)), dim3(256), 0, st, g->off, n, W.deg);
    GPM_LAUNCH_CHECK("k_degrees");
    hipLaunchKernelGGL(k_wedge_sum, dim3(grid_for(n, kBlock, 8)), dim3(kBlock), 0, st, W.deg, n,
                       W.sums->wedge);
    GPM_LAUNCH_CHECK("k_wedge_sum");
    gpm_status rc;
    if (k == 3) {
        rc = clique_run(g, 3, false, W.shared, W.shared_bytes, &W.sums->tri, nullptr, 0, nullptr,
                        st);
        if (rc) return rc;
    } else {
        if (g->m > 0) GPM_HIP(fill_u32(W.te, 0, (uint64_t)g->m, st));
        rc = triangle_arc_counts(g, W.shared, W.shared_bytes, W.te, &W.sums->tri, st);
        if (rc) return rc;
        if (g->m > 0) {
            hipLaunchKernelGGL(k_lc_sums, dim3(grid_for(g->m, kBlock, 8)), dim3(kBlock), 0, st,
                               g->dag_src, g->dag_adj, W.te, W.deg, g->m, W.sums->lc);
            GPM_LAUNCH_CHECK("k_lc_sums");
        }
        rc = clique_run(g, 4, false, W.shared, W.shared_bytes, &W.sums->k4, nullptr, 0, nullptr,
                        st);
        if (rc) return rc;
        rc = c4_run(g, false, W.c4ws, W.c4_bytes, W.sums->c4, nullptr, 0, nullptr, st);
        if (rc) return rc;
    }
    hipLaunchKernelGGL(k_combine, dim3(1), dim3(64), 0, st, W.sums, k, d_counts);
    GPM_LAUNCH_CHECK("k_combine");
    return GPM_OK;
}

}  // namespace gpm
