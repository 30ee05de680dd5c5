// The C ABI (include/gpm.h): argument validation, plan selection and
// dispatch.  Host code only; kernels live in the .hip translation units.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <string>

#include "gpm_internal.h"

namespace gpm {
gpm_status graph_build_bytes(int32_t n, int64_t E, uint64_t *gb, uint64_t *sb);
gpm_status clique_multi_workspace_bytes(const gpm_graph *g, int32_t kmax, uint64_t *bytes);
gpm_status clique_multi_run(const gpm_graph *g, int32_t kmax, void *ws, uint64_t ws_bytes,
                            unsigned long long *d_counts, hipStream_t st);
gpm_status graph_from_csr_bytes(int32_t n, int64_t nnz, uint64_t *gb, uint64_t *sb);
gpm_status graph_from_csr(int32_t n, const int32_t *d_off, const int32_t *d_adj, int64_t nnz,
                          int32_t validate, void *gmem, uint64_t gbytes, void *smem,
                          uint64_t sbytes, hipStream_t st, gpm_graph **out);
gpm_status graph_build(int32_t n, const int32_t *d_u, const int32_t *d_v, int64_t E, void *gmem,
                       uint64_t gbytes, void *smem, uint64_t sbytes, hipStream_t st,
                       gpm_graph **out);
gpm_status clique_workspace_bytes(const gpm_graph *g, int32_t k, bool list, uint64_t *bytes);
gpm_status clique_run(const gpm_graph *g, int32_t k, bool list, void *ws, uint64_t ws_bytes,
                      unsigned long long *d_count, int32_t *d_buf, uint64_t cap,
                      unsigned long long *d_result, hipStream_t st);
gpm_status motif_workspace_bytes(const gpm_graph *g, int32_t k, uint64_t *bytes);
gpm_status motif_run(const gpm_graph *g, int32_t k, void *ws, uint64_t ws_bytes,
                     unsigned long long *d_counts, hipStream_t st);
gpm_status sl_workspace_bytes(const gpm_graph *g, int32_t plan, bool list, uint64_t *bytes);
bool generic_pattern_ok(const gpm_pattern *p);
gpm_status generic_describe(const gpm_pattern *p, int32_t *order, uint32_t *less);
uint64_t generic_workspace_bytes(const gpm_graph *g);
gpm_status generic_list(const gpm_graph *g, const gpm_pattern *p, void *ws, uint64_t ws_bytes,
                        int32_t *buf, uint64_t cap, unsigned long long *result, hipStream_t st);
gpm_status generic_count(const gpm_graph *g, const gpm_pattern *p, void *ws, uint64_t ws_bytes,
                         unsigned long long *out, hipStream_t st);
gpm_status permute_rows4(int32_t *buf, uint64_t cap, const unsigned long long *result,
                         const int32_t perm[4], hipStream_t st);
gpm_status sl_run(const gpm_graph *g, int32_t plan, bool list, void *ws, uint64_t ws_bytes,
                  unsigned long long *d_count, int32_t *d_buf, uint64_t cap,
                  unsigned long long *d_result, hipStream_t st);
uint64_t orient_scratch_bytes(const gpm_graph *g);
void tuning_get(const gpm_graph *g, gpm_tuning *t);
gpm_status tuning_set(gpm_graph *g, const gpm_tuning *t);
gpm_status autotune_bytes(const gpm_graph *g, uint64_t *bytes);
gpm_status graph_autotune(gpm_graph *g, void *ws, uint64_t ws_bytes, hipStream_t st,
                          gpm_tuning *chosen);
gpm_status graph_orient(gpm_graph *g, int32_t order, void *scratch, uint64_t scratch_bytes,
                        int32_t *d_core, hipStream_t st);
int motif_classes(int k);
gpm_status motif_class_pattern(int k, int idx, gpm_pattern *out);
gpm_status motif_enum_workspace_bytes(const gpm_graph *g, uint64_t *bytes);
gpm_status motif_enum_count(const gpm_graph *g, int k, void *ws, uint64_t ws_bytes,
                            unsigned long long *out, hipStream_t st);
gpm_status motif_formula_workspace_bytes(const gpm_graph *g, int32_t k, uint64_t *bytes);
gpm_status motif_formula_count(const gpm_graph *g, int32_t k, void *ws, uint64_t ws_bytes,
                               unsigned long long *d_counts, hipStream_t st);
gpm_status batch_workspace_bytes(int32_t G, int32_t k, uint64_t *bytes);
gpm_status batch_default_config(gpm_batch_config *c);
gpm_status batch_run(const gpm_graph *g, const int32_t *d_voff, int32_t G, int32_t k,
                     const gpm_batch_config *cfg, void *ws, uint64_t ws_bytes,
                     unsigned long long *d_counts, hipStream_t st);
gpm_status batch_run_static(const gpm_graph *g, const int32_t *d_voff, int32_t G, int32_t k,
                            unsigned long long *d_counts, hipStream_t st);
gpm_status batch_autotune(const gpm_graph *g, const int32_t *d_voff, int32_t G, int32_t k,
                          void *ws, uint64_t ws_bytes, unsigned long long *d_counts,
                          hipStream_t st, int32_t reps, gpm_batch_config *best, float *best_ms);
}  // namespace gpm

using gpm::fail;

namespace {

bool aligned256(const void *p) { return ((uintptr_t)p & 255u) == 0; }

bool connected_pattern(int32_t k, int32_t ne, const int32_t (*e)[2]) {
    uint32_t reach = 1u;
    for (int it = 0; it < k; it++)
        for (int i = 0; i < ne; i++) {
            uint32_t a = 1u << e[i][0], b = 1u << e[i][1];
            if ((reach & a) || (reach & b)) reach |= a | b;
        }
    return reach == (k >= 32 ? ~0u : ((1u << k) - 1u));
}

// Degree sequence signature used to recognise patterns up to isomorphism for
// the patterns this library plans: with 4 vertices, (edge count, sorted
// degrees) separates all connected graphs.
void degree_sig(const gpm_pattern *p, int32_t *deg) {
    for (int i = 0; i < GPM_MAX_PATTERN_VERTICES; i++) deg[i] = 0;
    for (int i = 0; i < p->n_edges; i++) {
        deg[p->edges[i][0]]++;
        deg[p->edges[i][1]]++;
    }
}

gpm_status check_graph(const gpm_graph *g) {
    if (!g) return fail(GPM_INVALID_ARGUMENT, "graph is NULL");
    return GPM_OK;
}

// The subgraph-listing kernels write a diamond as (a, b, c, d) with a-b its
// diagonal and a 4-cycle in cycle order, i.e. as maps of these labelled
// patterns.  For the caller's labelling P of the same shape, perm[p] is the
// column of the kernel's row that holds pattern vertex p of P: an
// isomorphism phi from P onto the kernel's pattern (every edge (a, b) of P
// lands on an edge (phi(a), phi(b))), found by trying the 24 orders.
void sl_column_perm(const gpm_pattern *p, int32_t plan, int32_t perm[4]) {
    static const int32_t kDiamond[5][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}};
    static const int32_t kCycle[4][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 0}};
    bool q[4][4] = {};
    const int32_t (*qe)[2] = plan == GPM_PLAN_SL_DIAMOND ? kDiamond : kCycle;
    const int nq = plan == GPM_PLAN_SL_DIAMOND ? 5 : 4;
    for (int i = 0; i < nq; i++) q[qe[i][0]][qe[i][1]] = q[qe[i][1]][qe[i][0]] = true;
    int32_t phi[4] = {0, 1, 2, 3};
    do {
        bool ok = true;
        for (int i = 0; i < p->n_edges && ok; i++) ok = q[phi[p->edges[i][0]]][phi[p->edges[i][1]]];
        if (ok) break;
    } while (std::next_permutation(phi, phi + 4));
    for (int i = 0; i < 4; i++) perm[i] = phi[i];
}

}  // namespace

extern "C" {

const char *gpm_status_string(gpm_status s) {
    switch (s) {
        case GPM_OK: return "GPM_OK";
        case GPM_INVALID_ARGUMENT: return "GPM_INVALID_ARGUMENT";
        case GPM_OUT_OF_MEMORY: return "GPM_OUT_OF_MEMORY";
        case GPM_DEVICE_ERROR: return "GPM_DEVICE_ERROR";
        case GPM_TRUNCATED: return "GPM_TRUNCATED";
        case GPM_UNSUPPORTED: return "GPM_UNSUPPORTED";
        case GPM_NOT_CANONICAL: return "GPM_NOT_CANONICAL";
        case GPM_INCONSISTENT: return "GPM_INCONSISTENT";
        default: return "GPM_UNKNOWN_STATUS";
    }
}

const char *gpm_last_error(void) { return gpm::last_error().c_str(); }

const char *gpm_version(void) { return "gpmhip 0.1 gfx950"; }

gpm_status gpm_timing_enable(int32_t on) {
    gpm::timing_set(on != 0);
    return GPM_OK;
}

int32_t gpm_timing_read(const char **names, float *ms, uint64_t *units, int32_t cap) {
    return gpm::timing_read(names, ms, units, cap < 0 ? 0 : cap);
}

gpm_status gpm_pattern_from_edges(int32_t k, int32_t n_edges, const int32_t *uv, uint32_t flags,
                                  gpm_pattern *out) {
    if (!out) return fail(GPM_INVALID_ARGUMENT, "out is NULL");
    if (k < 2 || k > GPM_MAX_PATTERN_VERTICES)
        return fail(GPM_INVALID_ARGUMENT, "pattern size k must be in [2, 9]");
    if (n_edges < k - 1 || n_edges > k * (k - 1) / 2 || (n_edges > 0 && !uv))
        return fail(GPM_INVALID_ARGUMENT, "edge count impossible for a connected pattern");
    uint32_t ind = flags & (GPM_VERTEX_INDUCED | GPM_EDGE_INDUCED);
    if (ind != GPM_VERTEX_INDUCED && ind != GPM_EDGE_INDUCED)
        return fail(GPM_INVALID_ARGUMENT, "exactly one of GPM_VERTEX_INDUCED, GPM_EDGE_INDUCED");
    if (flags & ~(GPM_VERTEX_INDUCED | GPM_EDGE_INDUCED | GPM_LIST))
        return fail(GPM_INVALID_ARGUMENT, "unknown pattern flag");
    gpm_pattern p;
    std::memset(&p, 0, sizeof(p));
    p.k = k;
    p.n_edges = n_edges;
    p.flags = flags;
    bool seen[GPM_MAX_PATTERN_VERTICES][GPM_MAX_PATTERN_VERTICES] = {};
    for (int32_t i = 0; i < n_edges; i++) {
        int32_t a = uv[2 * i], b = uv[2 * i + 1];
        if (a < 0 || b < 0 || a >= k || b >= k || a == b)
            return fail(GPM_INVALID_ARGUMENT, "pattern edge endpoint out of range or a loop");
        int32_t lo = a < b ? a : b, hi = a < b ? b : a;
        if (seen[lo][hi]) return fail(GPM_INVALID_ARGUMENT, "repeated pattern edge");
        seen[lo][hi] = true;
        p.edges[i][0] = a;
        p.edges[i][1] = b;
    }
    if (!connected_pattern(k, n_edges, p.edges))
        return fail(GPM_INVALID_ARGUMENT, "pattern is not connected (connected patterns only)");
    *out = p;
    return GPM_OK;
}

gpm_status gpm_pattern_clique(int32_t k, uint32_t flags, gpm_pattern *out) {
    if (k < 2 || k > GPM_MAX_PATTERN_VERTICES)
        return fail(GPM_INVALID_ARGUMENT, "clique size must be in [2, 9]");
    int32_t uv[GPM_MAX_PATTERN_EDGES * 2];
    int32_t ne = 0;
    for (int32_t a = 0; a < k; a++)
        for (int32_t b = a + 1; b < k; b++) {
            uv[2 * ne] = a;
            uv[2 * ne + 1] = b;
            ne++;
        }
    return gpm_pattern_from_edges(k, ne, uv, flags, out);
}

gpm_status gpm_pattern_plan(const gpm_pattern *p, int32_t *plan) {
    if (!p || !plan) return fail(GPM_INVALID_ARGUMENT, "NULL argument");
    const int32_t k = p->k, ne = p->n_edges;
    // the struct may come from the caller directly: check it as
    // gpm_pattern_from_edges would before reading its edges
    if (k < 2 || k > GPM_MAX_PATTERN_VERTICES || ne < k - 1 || ne > k * (k - 1) / 2)
        return fail(GPM_INVALID_ARGUMENT, "pattern size or edge count out of range");
    const uint32_t ind = p->flags & (GPM_VERTEX_INDUCED | GPM_EDGE_INDUCED);
    if (ind != GPM_VERTEX_INDUCED && ind != GPM_EDGE_INDUCED)
        return fail(GPM_INVALID_ARGUMENT, "exactly one of GPM_VERTEX_INDUCED, GPM_EDGE_INDUCED");
    if (p->flags & ~(GPM_VERTEX_INDUCED | GPM_EDGE_INDUCED | GPM_LIST))
        return fail(GPM_INVALID_ARGUMENT, "unknown pattern flag");
    bool seen[GPM_MAX_PATTERN_VERTICES][GPM_MAX_PATTERN_VERTICES] = {};
    for (int32_t i = 0; i < ne; i++) {
        const int32_t a = p->edges[i][0], b = p->edges[i][1];
        if (a < 0 || b < 0 || a >= k || b >= k || a == b)
            return fail(GPM_INVALID_ARGUMENT, "pattern edge endpoint out of range or a loop");
        const int32_t lo = a < b ? a : b, hi = a < b ? b : a;
        if (seen[lo][hi]) return fail(GPM_INVALID_ARGUMENT, "repeated pattern edge");
        seen[lo][hi] = true;
    }
    if (!connected_pattern(k, ne, p->edges))
        return fail(GPM_INVALID_ARGUMENT, "pattern is not connected (connected patterns only)");
    const bool vertex_induced = (p->flags & GPM_VERTEX_INDUCED) != 0;
    // Orientation iff the pattern is a clique, |E| = |V|(|V|-1)/2; for a
    // clique, vertex- and edge-induced embeddings coincide.
    if (ne == k * (k - 1) / 2 && k >= 3) {
        if (k > 9) return fail(GPM_UNSUPPORTED, "cliques up to 9 vertices");
        *plan = GPM_PLAN_CLIQUE_DAG;
        return GPM_OK;
    }
    if (k == 4 && !vertex_induced) {
        int32_t d[GPM_MAX_PATTERN_VERTICES];
        degree_sig(p, d);
        int deg2 = 0, deg3 = 0;
        for (int i = 0; i < 4; i++) {
            deg2 += d[i] == 2;
            deg3 += d[i] == 3;
        }
        if (ne == 5 && deg3 == 2 && deg2 == 2) { *plan = GPM_PLAN_SL_DIAMOND; return GPM_OK; }
        if (ne == 4 && deg2 == 4) { *plan = GPM_PLAN_SL_4CYCLE; return GPM_OK; }
    }
    if (!gpm::generic_pattern_ok(p)) return GPM_UNSUPPORTED;   // error text set by the check
    *plan = GPM_PLAN_GENERIC;
    return GPM_OK;
}

gpm_status gpm_pattern_matching_order(const gpm_pattern *p, int32_t *order, uint32_t *less) {
    if (!p || !order || !less) return fail(GPM_INVALID_ARGUMENT, "NULL argument");
    int32_t plan;
    gpm_status rc = gpm_pattern_plan(p, &plan);
    if (rc) return rc;
    if (plan != GPM_PLAN_GENERIC)
        return fail(GPM_UNSUPPORTED, "the pattern is not on the general plan");
    return gpm::generic_describe(p, order, less);
}

gpm_status gpm_graph_build_bytes(int32_t n, int64_t n_input_edges, uint64_t *graph_bytes,
                                 uint64_t *scratch_bytes) {
    if (!graph_bytes || !scratch_bytes) return fail(GPM_INVALID_ARGUMENT, "NULL size pointer");
    return gpm::graph_build_bytes(n, n_input_edges, graph_bytes, scratch_bytes);
}

gpm_status gpm_graph_build(int32_t n, const int32_t *d_u, const int32_t *d_v,
                           int64_t n_input_edges, void *d_graph_mem, uint64_t graph_bytes,
                           void *d_scratch, uint64_t scratch_bytes, void *stream,
                           gpm_graph **out) {
    return gpm::graph_build(n, d_u, d_v, n_input_edges, d_graph_mem, graph_bytes, d_scratch,
                            scratch_bytes, static_cast<hipStream_t>(stream), out);
}

gpm_status gpm_graph_from_csr_bytes(int32_t n, int64_t nnz, uint64_t *graph_bytes,
                                    uint64_t *scratch_bytes) {
    if (!graph_bytes || !scratch_bytes) return fail(GPM_INVALID_ARGUMENT, "NULL argument");
    return gpm::graph_from_csr_bytes(n, nnz, graph_bytes, scratch_bytes);
}

gpm_status gpm_graph_from_csr(int32_t n, const int32_t *d_offsets, const int32_t *d_adj,
                              int64_t nnz, int32_t validate, void *d_graph_mem,
                              uint64_t graph_bytes, void *d_scratch, uint64_t scratch_bytes,
                              void *stream, gpm_graph **out) {
    return gpm::graph_from_csr(n, d_offsets, d_adj, nnz, validate, d_graph_mem, graph_bytes,
                               d_scratch, scratch_bytes, static_cast<hipStream_t>(stream), out);
}

gpm_status gpm_graph_get_info(const gpm_graph *g, gpm_graph_info *info) {
    if (!g || !info) return fail(GPM_INVALID_ARGUMENT, "NULL argument");
    info->n = g->n;
    info->m = g->m;
    info->max_degree = g->max_degree;
    info->max_out_degree = g->max_out_degree;
    info->reserved = 0;
    info->off = g->off;
    info->adj = g->adj;
    info->dag_off = g->dag_off;
    info->dag_adj = g->dag_adj;
    info->dag_src = g->dag_src;
    return GPM_OK;
}

void gpm_graph_release(gpm_graph *g) { delete g; }

gpm_status gpm_graph_orient_bytes(const gpm_graph *g, uint64_t *scratch_bytes) {
    gpm_status rc = check_graph(g);
    if (rc) return rc;
    if (!scratch_bytes) return fail(GPM_INVALID_ARGUMENT, "NULL argument");
    *scratch_bytes = gpm::orient_scratch_bytes(g);
    return GPM_OK;
}

gpm_status gpm_graph_orient(gpm_graph *g, int32_t order, void *d_scratch, uint64_t scratch_bytes,
                            int32_t *d_core, void *stream) {
    gpm_status rc = check_graph(g);
    if (rc) return rc;
    if (order != GPM_ORIENT_DEGREE && order != GPM_ORIENT_CORE)
        return fail(GPM_INVALID_ARGUMENT, "order must be GPM_ORIENT_DEGREE or GPM_ORIENT_CORE");
    if (!d_scratch || !aligned256(d_scratch))
        return fail(GPM_INVALID_ARGUMENT, "scratch NULL or unaligned");
    return gpm::graph_orient(g, order, d_scratch, scratch_bytes, d_core,
                             static_cast<hipStream_t>(stream));
}

gpm_status gpm_graph_get_tuning(const gpm_graph *g, gpm_tuning *t) {
    gpm_status rc = check_graph(g);
    if (rc) return rc;
    if (!t) return fail(GPM_INVALID_ARGUMENT, "NULL argument");
    gpm::tuning_get(g, t);
    return GPM_OK;
}

gpm_status gpm_graph_set_tuning(gpm_graph *g, const gpm_tuning *t) {
    gpm_status rc = check_graph(g);
    if (rc) return rc;
    if (!t) return fail(GPM_INVALID_ARGUMENT, "NULL argument");
    return gpm::tuning_set(g, t);
}

gpm_status gpm_graph_autotune_bytes(const gpm_graph *g, uint64_t *bytes) {
    gpm_status rc = check_graph(g);
    if (rc) return rc;
    if (!bytes) return fail(GPM_INVALID_ARGUMENT, "NULL argument");
    return gpm::autotune_bytes(g, bytes);
}

gpm_status gpm_graph_autotune(gpm_graph *g, void *d_ws, uint64_t ws_bytes, void *stream,
                              gpm_tuning *chosen) {
    gpm_status rc = check_graph(g);
    if (rc) return rc;
    if (!d_ws || !aligned256(d_ws)) return fail(GPM_INVALID_ARGUMENT, "workspace NULL or unaligned");
    return gpm::graph_autotune(g, d_ws, ws_bytes, static_cast<hipStream_t>(stream), chosen);
}

gpm_status gpm_workspace_bytes(const gpm_graph *g, const gpm_pattern *p, uint64_t *bytes) {
    gpm_status rc = check_graph(g);
    if (rc) return rc;
    if (!p || !bytes) return fail(GPM_INVALID_ARGUMENT, "NULL argument");
    int32_t plan;
    rc = gpm_pattern_plan(p, &plan);
    if (rc) return rc;
    const bool list = (p->flags & GPM_LIST) != 0;
    if (plan == GPM_PLAN_CLIQUE_DAG) return gpm::clique_workspace_bytes(g, p->k, list, bytes);
    if (plan == GPM_PLAN_GENERIC) {
        *bytes = gpm::generic_workspace_bytes(g);
        return GPM_OK;
    }
    return gpm::sl_workspace_bytes(g, plan, list, bytes);
}

gpm_status gpm_count(const gpm_graph *g, const gpm_pattern *p, void *d_ws, uint64_t ws_bytes,
                     uint64_t *d_count, void *stream) {
    gpm_status rc = check_graph(g);
    if (rc) return rc;
    if (!p || !d_count) return fail(GPM_INVALID_ARGUMENT, "NULL argument");
    if (p->flags & GPM_LIST) return fail(GPM_INVALID_ARGUMENT, "gpm_count with a GPM_LIST pattern");
    if (!d_ws || !aligned256(d_ws)) return fail(GPM_INVALID_ARGUMENT, "workspace NULL or unaligned");
    int32_t plan;
    rc = gpm_pattern_plan(p, &plan);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    unsigned long long *out = reinterpret_cast<unsigned long long *>(d_count);
    if (plan == GPM_PLAN_CLIQUE_DAG)
        return gpm::clique_run(g, p->k, false, d_ws, ws_bytes, out, nullptr, 0, nullptr, st);
    if (plan == GPM_PLAN_GENERIC) return gpm::generic_count(g, p, d_ws, ws_bytes, out, st);
    return gpm::sl_run(g, plan, false, d_ws, ws_bytes, out, nullptr, 0, nullptr, st);
}

gpm_status gpm_list(const gpm_graph *g, const gpm_pattern *p, void *d_ws, uint64_t ws_bytes,
                    int32_t *d_buf, uint64_t cap, uint64_t *d_result, void *stream) {
    gpm_status rc = check_graph(g);
    if (rc) return rc;
    if (!p || !d_result) return fail(GPM_INVALID_ARGUMENT, "NULL argument");
    if (!(p->flags & GPM_LIST)) return fail(GPM_INVALID_ARGUMENT, "gpm_list needs GPM_LIST");
    if (cap > 0 && !d_buf) return fail(GPM_INVALID_ARGUMENT, "cap > 0 with a NULL buffer");
    if (!d_ws || !aligned256(d_ws)) return fail(GPM_INVALID_ARGUMENT, "workspace NULL or unaligned");
    int32_t plan;
    rc = gpm_pattern_plan(p, &plan);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    unsigned long long *res = reinterpret_cast<unsigned long long *>(d_result);
    if (plan == GPM_PLAN_CLIQUE_DAG)
        return gpm::clique_run(g, p->k, true, d_ws, ws_bytes, nullptr, d_buf, cap, res, st);
    if (plan == GPM_PLAN_GENERIC)
        return gpm::generic_list(g, p, d_ws, ws_bytes, d_buf, cap, res, st);
    rc = gpm::sl_run(g, plan, true, d_ws, ws_bytes, nullptr, d_buf, cap, res, st);
    if (rc) return rc;
    int32_t perm[4];
    sl_column_perm(p, plan, perm);
    if (perm[0] == 0 && perm[1] == 1 && perm[2] == 2 && perm[3] == 3) return GPM_OK;
    return gpm::permute_rows4(d_buf, cap, res, perm, st);
}

gpm_status gpm_clique_counts_workspace_bytes(const gpm_graph *g, int32_t kmax, uint64_t *bytes) {
    gpm_status rc = check_graph(g);
    if (rc) return rc;
    if (!bytes) return fail(GPM_INVALID_ARGUMENT, "NULL argument");
    if (kmax != 4 && kmax != 5) return fail(GPM_UNSUPPORTED, "kmax must be 4 or 5");
    return gpm::clique_multi_workspace_bytes(g, kmax, bytes);
}

gpm_status gpm_clique_counts(const gpm_graph *g, int32_t kmax, void *d_ws, uint64_t ws_bytes,
                             uint64_t *d_counts, void *stream) {
    gpm_status rc = check_graph(g);
    if (rc) return rc;
    if (!d_counts) return fail(GPM_INVALID_ARGUMENT, "NULL argument");
    if (kmax != 4 && kmax != 5) return fail(GPM_UNSUPPORTED, "kmax must be 4 or 5");
    if (!d_ws || !aligned256(d_ws)) return fail(GPM_INVALID_ARGUMENT, "workspace NULL or unaligned");
    return gpm::clique_multi_run(g, kmax, d_ws, ws_bytes,
                                 reinterpret_cast<unsigned long long *>(d_counts),
                                 static_cast<hipStream_t>(stream));
}

gpm_status gpm_motif_workspace_bytes(const gpm_graph *g, int32_t k, uint64_t *bytes) {
    gpm_status rc = check_graph(g);
    if (rc) return rc;
    if (!bytes) return fail(GPM_INVALID_ARGUMENT, "NULL argument");
    if (k != 3 && k != 4) return fail(GPM_UNSUPPORTED, "motif size must be 3 or 4");
    return gpm::motif_workspace_bytes(g, k, bytes);
}

gpm_status gpm_motif_count(const gpm_graph *g, int32_t k, void *d_ws, uint64_t ws_bytes,
                           uint64_t *d_counts, void *stream) {
    gpm_status rc = check_graph(g);
    if (rc) return rc;
    if (!d_counts) return fail(GPM_INVALID_ARGUMENT, "NULL argument");
    if (k != 3 && k != 4) return fail(GPM_UNSUPPORTED, "motif size must be 3 or 4");
    if (!d_ws || !aligned256(d_ws)) return fail(GPM_INVALID_ARGUMENT, "workspace NULL or unaligned");
    return gpm::motif_run(g, k, d_ws, ws_bytes, reinterpret_cast<unsigned long long *>(d_counts),
                          static_cast<hipStream_t>(stream));
}

int32_t gpm_motif_classes(int32_t k) { return gpm::motif_classes(k); }

gpm_status gpm_motif_class_pattern(int32_t k, int32_t index, gpm_pattern *out) {
    if (!out) return fail(GPM_INVALID_ARGUMENT, "NULL argument");
    return gpm::motif_class_pattern(k, index, out);
}

gpm_status gpm_motif_enum_workspace_bytes(const gpm_graph *g, int32_t k, uint64_t *bytes) {
    gpm_status rc = check_graph(g);
    if (rc) return rc;
    if (k < 3 || k > 5) return fail(GPM_UNSUPPORTED, "motif size must be 3, 4 or 5");
    if (!bytes) return fail(GPM_INVALID_ARGUMENT, "NULL argument");
    return gpm::motif_enum_workspace_bytes(g, bytes);
}

gpm_status gpm_motif_count_enum(const gpm_graph *g, int32_t k, void *d_ws, uint64_t ws_bytes,
                                uint64_t *d_counts, void *stream) {
    gpm_status rc = check_graph(g);
    if (rc) return rc;
    if (k < 3 || k > 5) return fail(GPM_UNSUPPORTED, "motif size must be 3, 4 or 5");
    if (!d_counts) return fail(GPM_INVALID_ARGUMENT, "NULL argument");
    if (!d_ws || !aligned256(d_ws)) return fail(GPM_INVALID_ARGUMENT, "workspace NULL or unaligned");
    return gpm::motif_enum_count(g, k, d_ws, ws_bytes,
                                 reinterpret_cast<unsigned long long *>(d_counts),
                                 static_cast<hipStream_t>(stream));
}

gpm_status gpm_motif_formula_workspace_bytes(const gpm_graph *g, int32_t k, uint64_t *bytes) {
    gpm_status rc = check_graph(g);
    if (rc) return rc;
    if (!bytes) return fail(GPM_INVALID_ARGUMENT, "NULL argument");
    return gpm::motif_formula_workspace_bytes(g, k, bytes);
}

gpm_status gpm_motif_count_formula(const gpm_graph *g, int32_t k, void *d_ws, uint64_t ws_bytes,
                                   uint64_t *d_counts, void *stream) {
    gpm_status rc = check_graph(g);
    if (rc) return rc;
    if (k != 5) return fail(GPM_UNSUPPORTED, "formula motif counting is for k = 5");
    if (!d_counts) return fail(GPM_INVALID_ARGUMENT, "NULL argument");
    if (!d_ws || !aligned256(d_ws)) return fail(GPM_INVALID_ARGUMENT, "workspace NULL or unaligned");
    return gpm::motif_formula_count(g, k, d_ws, ws_bytes,
                                    reinterpret_cast<unsigned long long *>(d_counts),
                                    static_cast<hipStream_t>(stream));
}

gpm_status gpm_batch_workspace_bytes(int32_t G, int32_t k, uint64_t *bytes) {
    if (!bytes) return fail(GPM_INVALID_ARGUMENT, "NULL argument");
    if (G < 1) return fail(GPM_INVALID_ARGUMENT, "G must be >= 1");
    if (k != 3 && k != 4) return fail(GPM_UNSUPPORTED, "motif size must be 3 or 4");
    return gpm::batch_workspace_bytes(G, k, bytes);
}

static gpm_status check_batch(const gpm_graph *g, const int32_t *d_voff, int32_t G, int32_t k,
                              void *d_ws, uint64_t *d_counts) {
    gpm_status rc = check_graph(g);
    if (rc) return rc;
    if (!d_voff || !d_counts) return fail(GPM_INVALID_ARGUMENT, "NULL argument");
    if (G < 1) return fail(GPM_INVALID_ARGUMENT, "G must be >= 1");
    if (k != 3 && k != 4) return fail(GPM_UNSUPPORTED, "motif size must be 3 or 4");
    if (!d_ws || !aligned256(d_ws)) return fail(GPM_INVALID_ARGUMENT, "workspace NULL or unaligned");
    return GPM_OK;
}

gpm_status gpm_batch_default_config(gpm_batch_config *out) {
    if (!out) return fail(GPM_INVALID_ARGUMENT, "NULL argument");
    return gpm::batch_default_config(out);
}

gpm_status gpm_batch_motif_count_config(const gpm_graph *g, const int32_t *d_voff, int32_t G,
                                        int32_t k, const gpm_batch_config *cfg, void *d_ws,
                                        uint64_t ws_bytes, uint64_t *d_counts, void *stream) {
    gpm_status rc = check_batch(g, d_voff, G, k, d_ws, d_counts);
    if (rc) return rc;
    if (!cfg) return fail(GPM_INVALID_ARGUMENT, "NULL argument");
    return gpm::batch_run(g, d_voff, G, k, cfg, d_ws, ws_bytes,
                          reinterpret_cast<unsigned long long *>(d_counts),
                          static_cast<hipStream_t>(stream));
}

gpm_status gpm_batch_motif_count(const gpm_graph *g, const int32_t *d_voff, int32_t G, int32_t k,
                                 void *d_ws, uint64_t ws_bytes, uint64_t *d_counts,
                                 void *stream) {
    gpm_batch_config cfg;
    gpm::batch_default_config(&cfg);
    return gpm_batch_motif_count_config(g, d_voff, G, k, &cfg, d_ws, ws_bytes, d_counts, stream);
}

gpm_status gpm_batch_motif_count_static(const gpm_graph *g, const int32_t *d_voff, int32_t G,
                                        int32_t k, uint64_t *d_counts, void *stream) {
    gpm_status rc = check_graph(g);
    if (rc) return rc;
    if (!d_voff || !d_counts) return fail(GPM_INVALID_ARGUMENT, "NULL argument");
    if (G < 1) return fail(GPM_INVALID_ARGUMENT, "G must be >= 1");
    if (k != 3 && k != 4) return fail(GPM_UNSUPPORTED, "motif size must be 3 or 4");
    return gpm::batch_run_static(g, d_voff, G, k, reinterpret_cast<unsigned long long *>(d_counts),
                                 static_cast<hipStream_t>(stream));
}

gpm_status gpm_batch_autotune(const gpm_graph *g, const int32_t *d_voff, int32_t G, int32_t k,
                              void *d_ws, uint64_t ws_bytes, uint64_t *d_counts, void *stream,
                              int32_t reps, gpm_batch_config *best, float *best_ms) {
    gpm_status rc = check_batch(g, d_voff, G, k, d_ws, d_counts);
    if (rc) return rc;
    if (!best) return fail(GPM_INVALID_ARGUMENT, "NULL argument");
    if (reps < 1) return fail(GPM_INVALID_ARGUMENT, "reps must be >= 1");
    return gpm::batch_autotune(g, d_voff, G, k, d_ws, ws_bytes,
                               reinterpret_cast<unsigned long long *>(d_counts),
                               static_cast<hipStream_t>(stream), reps, best, best_ms);
}

}  // extern "C"
