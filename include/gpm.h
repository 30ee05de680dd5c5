/*
 * gpm.h -- C ABI of the MI355X (gfx950) graph pattern mining library
 * (libgpmhip.so).
 *
 * What it computes.  Given an undirected graph G and a pattern P (Section 2,
 * problem definition; Section 3.1, high-level API: induced-ness flag,
 * listing-or-counting flag, explicit pattern edge list, runtime size k), the
 * library counts or lists the embeddings of P in G:
 *   - triangle counting and k-clique counting/listing (problems 1-2),
 *     vertex-induced, on the degree-ordered DAG (Appendix B.2);
 *   - subgraph listing of the diamond and the 4-cycle, edge-induced
 *     (problem 3; matching order and partial orders of Appendices B.1, B.3);
 *   - k-motif counting for k = 3, 4, vertex-induced, connected patterns only
 *     (problem 4), by local counting (Section 5, the wedge equation; the
 *     3-motif and 4-motif local-counting listings of Appendix A);
 *   - k-motif counting for k = 3, 4, 5 by pattern-oblivious enumeration
 *     (Section 4: vertex extension, connectivity codes);
 *   - the same motif counts for a batch of small graphs in one launch.
 *
 * Conventions shared by every entry point.
 *   - No entry point throws, aborts or exits on bad input; each returns a
 *     gpm_status.  gpm_last_error() (thread-local) describes the last
 *     failure on the calling thread.
 *   - Device memory is owned by the caller: every device buffer (inputs,
 *     outputs, graph storage, workspace) is allocated and freed by the
 *     caller.  The library performs no device allocation in any entry point.
 *     Required sizes come from the *_bytes query functions.  Every device
 *     pointer must be 256-byte aligned.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Work is
 *     enqueued asynchronously on it; outputs are valid once the stream has
 *     been synchronised.  Exceptions are stated per function (gpm_graph_build
 *     synchronises the stream once, to learn the graph's sizes).
 *   - Argument errors are detected on the host before anything is enqueued.
 *     HIP errors are returned as GPM_DEVICE_ERROR.
 *   - Vertex ids are int32 in [0, n).  The symmetric adjacency must have
 *     fewer than 2^31 entries.  Counts are exact uint64.
 *   - Calls that share a workspace buffer must not overlap in time (same
 *     stream, or the caller orders them).  Graph storage is read-only after
 *     gpm_graph_build and may be shared by concurrent calls.
 */
#ifndef GPM_H
#define GPM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status --- */

typedef int32_t gpm_status;
#define GPM_OK                0
#define GPM_INVALID_ARGUMENT  1  /* bad pointer, size, id or flag combination */
#define GPM_OUT_OF_MEMORY     2  /* a caller buffer is smaller than required */
#define GPM_DEVICE_ERROR      3  /* a HIP call failed; see gpm_last_error() */
#define GPM_TRUNCATED         4  /* (reported in listing results, see gpm_list) */
#define GPM_UNSUPPORTED       5  /* pattern or size outside what is implemented */
#define GPM_NOT_CANONICAL     6  /* input not in the required form (ids out of range, a
                                    failed CSR check) */
#define GPM_INCONSISTENT      7  /* an exact-division check of a formula failed */

/* Static string naming a status code. */
const char *gpm_status_string(gpm_status s);
/* Description of the last failure on the calling thread ("" if none). */
const char *gpm_last_error(void);
/* Library version string, e.g. "gpmhip 0.1 gfx950". */
const char *gpm_version(void);

/* ----------------------------------------------------------- pattern --- */

/* Pattern flags (Section 3.1: the two required per-problem flags). */
#define GPM_VERTEX_INDUCED 0x1u
#define GPM_EDGE_INDUCED   0x2u
#define GPM_LIST           0x4u   /* listing; absent means counting */

#define GPM_MAX_PATTERN_VERTICES 9
#define GPM_MAX_PATTERN_EDGES    36

/* A pattern is an edge list on vertices 0..k-1 (Section 3.1: patterns are
 * given as edge lists, e.g. the triangle {(0,1),(0,2),(1,2)}). */
typedef struct gpm_pattern {
    int32_t k;                                   /* number of vertices */
    int32_t n_edges;                             /* number of edges */
    int32_t edges[GPM_MAX_PATTERN_EDGES][2];     /* pairs (a, b), a != b */
    uint32_t flags;                              /* exactly one of *_INDUCED, optional GPM_LIST */
} gpm_pattern;

/* Builds the pattern from an edge list (uv holds n_edges pairs, host
 * memory).  Rejects loops, repeated edges, ids outside [0, k), disconnected
 * patterns and k outside [2, 9] with GPM_INVALID_ARGUMENT. */
gpm_status gpm_pattern_from_edges(int32_t k, int32_t n_edges, const int32_t *uv,
                                  uint32_t flags, gpm_pattern *out);
/* The k-clique (helper named in Section 3.1); flags as above. */
gpm_status gpm_pattern_clique(int32_t k, uint32_t flags, gpm_pattern *out);

/* Plan chosen for a pattern (Section 4.3 enablement rules: orientation
 * iff the pattern is a clique, |E| = |V|(|V|-1)/2 (Appendix B.2); a
 * matching order with partial orders for other single explicit patterns). */
/* Cliques of k >= 4 are searched on local graphs (Section 5) from roots of
 * out-degree up to 1024; roots above that (hubs) are split into one task
 * per out-arc (Section 4.1) and searched depth first below the arc.
 * GPM_LG=0 in the environment sends every root to the depth-first search
 * without local graphs instead (same results; for comparison). */
#define GPM_PLAN_CLIQUE_DAG     1   /* triangles and k-cliques, k <= 9 */
#define GPM_PLAN_SL_DIAMOND     2   /* edge-induced diamond listing/counting */
#define GPM_PLAN_SL_4CYCLE      3   /* edge-induced 4-cycle listing/counting */
/* Any other connected pattern of 2..6 vertices, vertex- or edge-induced,
 * counted or listed (gpm_list's conventions; each embedding once, written
 * as the data vertices of pattern vertices 0..k-1).  A matching order with
 * partial orders derived from the pattern's automorphisms (Appendix B.1);
 * waves take work units of 64 third-vertex candidates below one edge and
 * search depth first below each.  Patterns of up to 5 vertices on graphs of
 * up to 8192 vertices test adjacency through a per-wave connectivity map
 * in LDS (Section 4, memoised neighbourhood connectivity), others by binary
 * search in the matched vertices' rows; GPM_MNC=0 in the environment forces
 * the latter.  Both give the same counts. */
#define GPM_PLAN_GENERIC        4
/* How the general plan (GPM_PLAN_GENERIC) searches pattern p.  order[s]
 * (k entries) is the pattern vertex matched at step s: the greedy of
 * Appendix B.3 (each step adjacent to an earlier one; the sub-pattern with
 * more internal partial orders first, then the denser one; then the higher
 * degree, then the lower id; the first two steps an edge carrying a
 * partial order when one exists).  less[x] (k entries) is the set of
 * pattern vertices y (bit y) with f(x) < f(y) required of every match f:
 * the symmetry-breaking partial orders of Appendix B.1, from the stabiliser
 * chain of the automorphism group with vertices taken by degree (highest
 * first, then lowest id), so that each embedding is matched exactly once.
 * Every step also skips data vertices of smaller degree than its pattern
 * vertex (degree filtering, Section 4.3; GPM_DF=0 in the environment turns
 * it off, with the same results).  Host only.  GPM_UNSUPPORTED for patterns
 * on another plan. */
gpm_status gpm_pattern_matching_order(const gpm_pattern *p, int32_t *order, uint32_t *less);

/* Returns the plan for (graph-independent) pattern p, or GPM_UNSUPPORTED.
 * A struct built by the caller is checked as gpm_pattern_from_edges would
 * check it (sizes, edges, connectivity, and flags: exactly one of
 * GPM_VERTEX_INDUCED and GPM_EDGE_INDUCED, no unknown bit), else
 * GPM_INVALID_ARGUMENT.  Every counting and listing entry point runs this
 * check first. */
gpm_status gpm_pattern_plan(const gpm_pattern *p, int32_t *plan);

/* ------------------------------------------------------------- graph --- */

/* Opaque host handle.  It records device pointers into caller-owned graph
 * storage and the graph's sizes; it owns no device memory. */
typedef struct gpm_graph gpm_graph;

/* Sizes of the caller buffers gpm_graph_build needs for a graph on n
 * vertices given by n_input_edges raw edge-stream entries.  graph_bytes is
 * kept for the graph's lifetime; scratch_bytes only during the build.
 * n must be in [1, 2^31 - 2]; 2 * n_input_edges must be < 2^31. */
gpm_status gpm_graph_build_bytes(int32_t n, int64_t n_input_edges,
                                 uint64_t *graph_bytes, uint64_t *scratch_bytes);

/* Builds the canonical graph on the device from a raw undirected edge stream
 * (d_u[i], d_v[i]), i < n_input_edges (device int32 arrays): self-loops are
 * dropped, repeated and reversed pairs are merged, rows are sorted -- the
 * input form the method assumes (Section 6, input-graph table caption).  It
 * then orients the graph by degree: each edge points to the endpoint of
 * larger degree, ties to the larger id (Appendix B.2).  Stored in
 * d_graph_mem (graph_bytes, from gpm_graph_build_bytes):
 *   symmetric CSR  off int32[n+1], adj int32[2m], rows ascending;
 *   oriented CSR   dag_off int32[n+1], dag_adj int32[m], rows ascending;
 *                  arc index e in [0, m) is the undirected edge id;
 *   arc sources    dag_src int32[m].
 * d_scratch (scratch_bytes) may be reused once the call returns.  The call
 * synchronises `stream` once.  Ids outside [0, n) give GPM_NOT_CANONICAL
 * (and *out is not set).  On success *out must later be released with
 * gpm_graph_release. */
gpm_status gpm_graph_build(int32_t n, const int32_t *d_u, const int32_t *d_v,
                           int64_t n_input_edges, void *d_graph_mem, uint64_t graph_bytes,
                           void *d_scratch, uint64_t scratch_bytes, void *stream,
                           gpm_graph **out);

/* Sizes for gpm_graph_from_csr: a graph on n vertices whose symmetric CSR has
 * nnz = 2m entries.  nnz must be even and below 2^31. */
gpm_status gpm_graph_from_csr_bytes(int32_t n, int64_t nnz, uint64_t *graph_bytes,
                                    uint64_t *scratch_bytes);

/* Graph from a caller's symmetric CSR already in the method's input form
 * (Section 6, input-graph table caption): d_offsets int32[n+1] with
 * d_offsets[0] = 0 and d_offsets[n] = nnz, d_adj int32[nnz] (device).  Both
 * are copied into d_graph_mem (same layout as gpm_graph_build) and the graph
 * is oriented by degree (Appendix B.2).  Always checked on the device:
 * offsets ascending and consistent with nnz, ids in [0, n).  With
 * validate != 0 also: rows strictly ascending, no self-loops, every arc
 * present in both directions.  A failed check gives GPM_NOT_CANONICAL (*out
 * not set); with validate == 0 a graph outside the form gives undefined
 * counts.  Synchronises `stream` once. */
gpm_status gpm_graph_from_csr(int32_t n, const int32_t *d_offsets, const int32_t *d_adj,
                              int64_t nnz, int32_t validate, void *d_graph_mem,
                              uint64_t graph_bytes, void *d_scratch, uint64_t scratch_bytes,
                              void *stream, gpm_graph **out);

typedef struct gpm_graph_info {
    int32_t n;              /* vertices */
    int32_t max_degree;     /* largest undirected degree */
    int64_t m;              /* undirected edges after canonicalisation */
    int32_t max_out_degree; /* largest out-degree of the oriented graph */
    int32_t reserved;
    const int32_t *off, *adj, *dag_off, *dag_adj, *dag_src;   /* device */
} gpm_graph_info;

gpm_status gpm_graph_get_info(const gpm_graph *g, gpm_graph_info *info);
/* Frees the host handle (not the caller's device memory).  NULL is a no-op. */
void gpm_graph_release(gpm_graph *g);

/* Orientation of the graph's DAG (Appendix B.2: by degree, the build's
 * default, or by core value).  GPM_ORIENT_CORE computes every vertex's core
 * number (the largest k whose k-core holds it) and rebuilds the DAG with
 * arc u -> v iff (core(u), deg(u), u) < (core(v), deg(v), v), degrees
 * capped at 2^(31 - bits of the largest core) - 1; GPM_ORIENT_DEGREE
 * rebuilds the degree order (deg(u), u) < (deg(v), v).  The DAG arrays are rewritten in
 * place in the graph's storage and the handle's max_out_degree is updated;
 * counts do not depend on the orientation.  d_core (device int32[n], may be
 * NULL) receives the core numbers; they are computed (for d_core) under
 * either order.  Core numbers come from the h-index fixed point (each
 * vertex repeatedly takes the h-index of its neighbours' values, starting
 * from an upper bound; rounds queued 8 at a time); graphs whose bound
 * exceeds 4095 are peeled level by level instead (queued device steps).
 * d_scratch is only used during the call; the call synchronises the stream
 * (the host reads a few counters per batch through a 64-byte pinned host
 * buffer the first call allocates and the process keeps).  Must not run
 * while other work on the same graph is in flight. */
#define GPM_ORIENT_DEGREE 1
#define GPM_ORIENT_CORE   2
gpm_status gpm_graph_orient_bytes(const gpm_graph *g, uint64_t *scratch_bytes);
gpm_status gpm_graph_orient(gpm_graph *g, int32_t order, void *d_scratch, uint64_t scratch_bytes,
                            int32_t *d_core, void *stream);

/* Task granularity of the plain path, kept per graph handle (Section 4.1
 * splits the work into tasks and leaves their size open).  Triangle
 * counting (and the per-edge triangle counts of local counting) splits the
 * (root, out-neighbour) pair space of each out-degree class, (1, 64],
 * (64, 256] and (256, 1024], into chunks of tc_tau pairs that
 * cu_count * tc_blocks_per_cu persistent workgroups take from an atomic
 * cursor; 5-clique counting splits each root of out-degree above 256 into
 * tasks of about lg5_slice local triangles; k-cliques (k >= 4) at roots of
 * out-degree up to 64 are counted a wave per root, roots dealt round robin
 * to cu_count * clique_wave_blocks_per_cu one-wave workgroups.  Counts never
 * depend on these.  A new handle starts at tc_tau = {8192, 16384, 65536},
 * tc_blocks_per_cu = {32, 8, 4}, clique_wave_blocks_per_cu = 32,
 * lg5_slice = 2^20.  Workspace sizes depend on tc_tau: query
 * them after changing it (a workspace sized before a smaller tc_tau gives
 * GPM_OUT_OF_MEMORY). */
typedef struct gpm_tuning {
    int64_t tc_tau[3];            /* pairs per chunk, [2048, 2^24] */
    int32_t tc_blocks_per_cu[3];  /* workgroups per CU, [1, 64] */
    int32_t clique_wave_blocks_per_cu;   /* [8, 1024] */
    int64_t lg5_slice;            /* local triangles per task, [2^14, 2^28] */
} gpm_tuning;

/* Host only.  set: GPM_INVALID_ARGUMENT for a value outside its range (the
 * handle keeps its tuning). */
gpm_status gpm_graph_get_tuning(const gpm_graph *g, gpm_tuning *t);
gpm_status gpm_graph_set_tuning(gpm_graph *g, const gpm_tuning *t);

/* Autotuner: times triangle counting, 4-clique counting and (when the graph
 * has roots of out-degree above 256) 5-clique counting on g under candidate
 * settings, walking the knobs one at a time (each tc_tau x4, x2, /2, /4,
 * each tc_blocks_per_cu x2, /2, two passes; clique_wave_blocks_per_cu x4,
 * x2, /2; lg5_slice x4, x2, /2, /4) and
 * keeping a change when it is at least 3% faster (median of three calls
 * after a warm-up, HIP events on the stream).  Stores the result in the
 * handle and, when chosen is not NULL, in *chosen; on failure the handle
 * keeps the tuning it had.  d_ws: at least
 * gpm_graph_autotune_bytes bytes, 256-byte aligned; the call synchronises
 * the stream.  Must not run while other work on the same graph is in
 * flight. */
gpm_status gpm_graph_autotune_bytes(const gpm_graph *g, uint64_t *bytes);
gpm_status gpm_graph_autotune(gpm_graph *g, void *d_ws, uint64_t ws_bytes, void *stream,
                              gpm_tuning *chosen);

/* ------------------------------------------------- counting, listing --- */

/* Workspace needed by gpm_count / gpm_list for pattern p on graph g. */
gpm_status gpm_workspace_bytes(const gpm_graph *g, const gpm_pattern *p, uint64_t *bytes);

/* Counts the embeddings of p in g (Section 2: unique subgraphs, each
 * automorphism class once), by the plan gpm_pattern_plan picks:
 * triangles and k-cliques for k <= 9 (either induced flag: for a clique the
 * two coincide); edge-induced diamonds and 4-cycles; any other connected
 * pattern of 2..6 vertices, vertex- or edge-induced, by the general plan.
 * Writes one uint64 to d_count (device).  p must not carry GPM_LIST.  A
 * workspace smaller than gpm_workspace_bytes gives GPM_OUT_OF_MEMORY before
 * anything is enqueued (d_count untouched). */
gpm_status gpm_count(const gpm_graph *g, const gpm_pattern *p, void *d_ws, uint64_t ws_bytes,
                     uint64_t *d_count, void *stream);

/* Lists the embeddings of p in g: the patterns gpm_count counts, cliques
 * of k <= 9 included.  Embedding number i (in an unspecified order) is
 * written to d_buf[i*k .. i*k+k-1] as the data vertices matched to pattern
 * vertices 0..k-1 of p as the caller labelled it (every pattern edge (a, b)
 * lands on a graph edge), for i < cap.  d_result (device uint64[3])
 * receives {total, written, checksum}: total counts every embedding even
 * past cap, written = min(total, cap), and checksum is the sum modulo 2^64,
 * over all embeddings, of a per-embedding hash of its canonical key:
 *     h = L; for each key element c in ascending order:
 *         h = fmix64((h XOR c) + 0x9E3779B97F4A7C15)
 * (fmix64 = the splitmix64 finaliser), with key = the ascending vertex
 * tuple for vertex-induced patterns and for cliques (whose vertex- and
 * edge-induced embeddings are the same vertex sets), and the ascending edge
 * codes (min << 32 | max) for the other edge-induced patterns; L is the
 * key's length.  written < total means the listing was truncated
 * (GPM_TRUNCATED is not returned, since the call is asynchronous).  p must
 * carry GPM_LIST.  A workspace smaller than gpm_workspace_bytes gives
 * GPM_OUT_OF_MEMORY before anything is enqueued (outputs untouched). */
gpm_status gpm_list(const gpm_graph *g, const gpm_pattern *p, void *d_ws, uint64_t ws_bytes,
                    int32_t *d_buf, uint64_t cap, uint64_t *d_result, void *stream);

/* Triangles, 4-cliques and (kmax = 5) 5-cliques of g in one pass: the
 * local graph on N+(u) (Section 5, search on a local graph) holds the
 * triangles at root u as its edges, the 4-cliques at u as its triangles and
 * the 5-cliques at u as its 4-cliques, so one build per root serves every
 * size (the per-size calls of gpm_count build it once per size).  Writes
 * d_counts (device uint64[kmax - 2]) = {3-cliques, 4-cliques[, 5-cliques]},
 * the same values as gpm_count per size.  kmax must be 4 or 5.  Roots of
 * out-degree above 1024 (too large for the local graph in LDS) are split
 * into one task per out-arc and searched depth first below the arc, with
 * the same counts. */
gpm_status gpm_clique_counts_workspace_bytes(const gpm_graph *g, int32_t kmax, uint64_t *bytes);
gpm_status gpm_clique_counts(const gpm_graph *g, int32_t kmax, void *d_ws, uint64_t ws_bytes,
                             uint64_t *d_counts, void *stream);

/* ----------------------------------------------------------- motifs --- */

/* Workspace needed by gpm_motif_count(g, k). */
gpm_status gpm_motif_workspace_bytes(const gpm_graph *g, int32_t k, uint64_t *bytes);

/* Induced k-motif counts, k = 3 or 4 (problem 4, connected patterns only),
 * written to d_counts (device uint64) in this fixed order:
 *   k = 3: {wedge, triangle}, then a status word;
 *   k = 4: {3-star, 4-path, 4-cycle, tailed-triangle, diamond, 4-clique},
 *          then a status word.
 * The status word is 0 when every exact division of the combining formulas
 * held and every count fit in 64 bits, nonzero otherwise. */
gpm_status gpm_motif_count(const gpm_graph *g, int32_t k, void *d_ws, uint64_t ws_bytes,
                           uint64_t *d_counts, void *stream);

/* Pattern-oblivious motif counting (Section 4, high-level Sandslash: vertex
 * extension of canonical embeddings with memoised connectivity codes, each
 * finished embedding classified by its code; Section 2 problem 4).  Every
 * connected vertex-induced k-vertex subgraph is enumerated once, so the
 * cost grows with their number: this is the route without the
 * local-counting formulas, for k = 3, 4 (the same values as
 * gpm_motif_count) and for k = 5, which has no formula route here.
 *
 * gpm_motif_classes(k): the number of motif classes, 2, 6 or 21 for
 * k = 3, 4, 5 (0 otherwise).  gpm_motif_class_pattern(k, i, out): the
 * pattern of class i (vertex-induced flag set).  Classes of k = 3 and 4 are
 * in gpm_motif_count's order; those of k = 5 are ordered by edge count, then
 * by the canonical code (the smallest, over vertex orders, of the number
 * whose bit l(l-1)/2 + j is set iff pattern vertices j < l are adjacent).
 * Host only; GPM_UNSUPPORTED for k outside [3, 5], GPM_INVALID_ARGUMENT for
 * i outside [0, classes). */
int32_t gpm_motif_classes(int32_t k);
gpm_status gpm_motif_class_pattern(int32_t k, int32_t index, gpm_pattern *out);

/* Workspace needed by gpm_motif_count_enum(g, k): 12 bytes per arc of the
 * symmetric CSR plus a little (the work-unit numbering). */
gpm_status gpm_motif_enum_workspace_bytes(const gpm_graph *g, int32_t k, uint64_t *bytes);
/* Writes d_counts (device uint64[gpm_motif_classes(k)]) = the induced count
 * of every class, k = 3, 4 or 5.  GPM_UNSUPPORTED for other k.  For k >= 4
 * on graphs of at most 16384 vertices each wave keeps a connectivity map in
 * LDS (Section 4, memoised neighbourhood connectivity: 4 bits per vertex,
 * the positions of the embedding it is adjacent to); elsewhere, or with the
 * environment variable GPM_MNC=0, the same bits come from binary
 * searches in the embedding's rows.  Both give the same counts. */
gpm_status gpm_motif_count_enum(const gpm_graph *g, int32_t k, void *d_ws, uint64_t ws_bytes,
                                uint64_t *d_counts, void *stream);

/* Induced 5-motif counts by formulas (Section 7 names counting motifs by
 * formulas; the route follows ESCAPE, Pinar, Seshadhri and Vishal, WWW
 * 2017).  The non-induced count N(P) of every connected 5-vertex pattern --
 * the number of its copies as edge sets -- is obtained, then the induced
 * counts by exact back-substitution through N(P) = sum over H of
 * c(P, H) I(H), c(P, H) the spanning copies of P in H.  Fifteen N(P)
 * (the 4-star, chair, 5-path, cricket, bull, 4-cycle with a pendant,
 * tadpole, dart, diamond with a pendant at a tip, bowtie, house, 4-clique
 * with a pendant, three triangles on one edge, a vertex joined to a
 * 4-path, and a 4-clique with a vertex joined to two of it) come from
 * closed forms in local counts: degrees, per-edge triangle counts
 * (Section 5), per-vertex triangle counts, neighbour-degree sums, sums
 * over the triangles, the 4-cycles and the 4-cliques, and the numbers of
 * 4-cycles and 4-cliques.  On graphs of up to 65,536 vertices five more
 * come from the rows of A^2, the triangles and the neighbourhoods: the
 * 5-cycle's from closed walks,
 * [tr(A^5) - 30 T - 10 sum_v (d_v - 2) t_v] / 10 (T triangles, t_v
 * those at v), K_{2,3}'s as the sum over vertex pairs of C(common
 * neighbours, 3), that of two triangles on an edge whose tips share a
 * third neighbour from pairs and triangles, and K5 minus an edge's as the
 * sum over triangles of C(vertices adjacent to all three, 2), and the
 * wheel's as the sum over vertices of the 4-cycles among their neighbours;
 * on larger graphs the five are counted directly as vertex-induced
 * patterns by the general plan.  K5 is counted by the clique kernels.
 * Writes d_counts (device uint64[22]): the 21
 * classes in gpm_motif_class_pattern order (the same values as
 * gpm_motif_count_enum), then a status word, 0 when every subtraction
 * stayed non-negative and every count fits 64 bits.  k must be 5
 * (GPM_UNSUPPORTED otherwise). */
gpm_status gpm_motif_formula_workspace_bytes(const gpm_graph *g, int32_t k, uint64_t *bytes);
gpm_status gpm_motif_count_formula(const gpm_graph *g, int32_t k, void *d_ws, uint64_t ws_bytes,
                                   uint64_t *d_counts, void *stream);

/* ------------------------------------------------------------ batch --- */

/* Batched motif counting over G small graphs held as ONE graph g (their
 * disjoint union, built with gpm_graph_build from the concatenated edge
 * streams with vertex ids shifted per graph): graph i owns vertices
 * d_voff[i] .. d_voff[i+1]-1 (device int32[G+1], ascending, within [0, n];
 * d_voff needs only 4-byte alignment and may point into a longer offset
 * array, so any run of consecutive graphs of the union, one graph
 * included, can be mined on its own).  No edge may join two graphs.  Writes d_counts (device
 * uint64[G][k == 3 ? 3 : 7]) row i = gpm_motif_count's output for graph i:
 * the k = 3 or k = 4 induced motif counts (Section 2, motif counting; the
 * local-count identities of Section 5), then a status word: 0, or an OR of
 * 1 (an exact division of the identities failed), 64 (the graph has more
 * than GPM_BATCH_MAX_VERTICES vertices; counts 0), 128 (d_voff[i..i+1] not
 * an ascending range within [0, n]; counts 0), 256 (an edge leaves the
 * graph's range).  The workspace (gpm_batch_workspace_bytes, 256-byte
 * aligned) holds the order in which graphs are mined.  Nothing is
 * allocated and the host never waits, so the call can be captured in a HIP
 * graph. */
#define GPM_BATCH_MAX_VERTICES 1024
gpm_status gpm_batch_workspace_bytes(int32_t G, int32_t k, uint64_t *bytes);
gpm_status gpm_batch_motif_count(const gpm_graph *g, const int32_t *d_voff, int32_t G,
                                 int32_t k, void *d_ws, uint64_t ws_bytes,
                                 uint64_t *d_counts, void *stream);

/* gpm_batch_motif_count for callers that cannot allocate (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * the same computation, results and kernels, with the work area that
 * gpm_batch_motif_count takes as d_ws held instead in a static device array
 * of GPM_BATCH_STATIC_SCRATCH_BYTES that the library keeps on each device
 * it runs on until the process ends.  The caller passes inputs and outputs
 * only.  No memory of any kind is allocated (no timing spans are recorded
 * either).  G above GPM_BATCH_STATIC_MAX_GRAPHS gives GPM_OUT_OF_MEMORY
 * before anything is enqueued.  Calls on one device share that device's
 * array: calls that overlap in time on the same device (other streams,
 * other threads) race and must be ordered by the caller. */
#define GPM_BATCH_STATIC_SCRATCH_BYTES (4u << 20)
#define GPM_BATCH_STATIC_MAX_GRAPHS 1045492
gpm_status gpm_batch_motif_count_static(const gpm_graph *g, const int32_t *d_voff, int32_t G,
                                        int32_t k, uint64_t *d_counts, void *stream);

/* How a batch is mined.  Graphs are mined largest first by teams of
 * threads, one graph per team at a time, each graph's adjacency held as bit
 * rows in LDS.  Graphs of 257..1024 vertices always go to 256-thread teams;
 * for graphs of at most 256 vertices:
 *   team_threads   64, 128 or 256 threads per team;
 *   tiers          1: one launch sized for 256 vertices; 2: graphs of at
 *                  most 128 vertices get their own launch with 4x smaller
 *                  LDS rows; 3: also graphs of at most 64 vertices;
 *   blocks_per_cu  1..32 resident teams per compute unit requested. */
typedef struct {
    int32_t team_threads;
    int32_t tiers;
    int32_t blocks_per_cu;
    int32_t reserved;          /* 0 */
} gpm_batch_config;

/* The configuration gpm_batch_motif_count uses. */
gpm_status gpm_batch_default_config(gpm_batch_config *out);

/* gpm_batch_motif_count with an explicit configuration (INVALID_ARGUMENT
 * if a field is out of range). */
gpm_status gpm_batch_motif_count_config(const gpm_graph *g, const int32_t *d_voff, int32_t G,
                                        int32_t k, const gpm_batch_config *cfg, void *d_ws,
                                        uint64_t ws_bytes, uint64_t *d_counts, void *stream);

/* Autotuner: mines the batch once per candidate configuration (every
 * combination of team_threads {64, 128, 256}, tiers {1, 2, 3} and
 * blocks_per_cu {4, 8, 16, 32}) and then `reps` more times timed with HIP
 * events on `stream`, keeps the fastest, and leaves d_counts as that
 * configuration computed them (every configuration computes the same
 * counts).  Blocks the calling thread (it waits for the stream); not for use
 * under graph capture.  *best_ms (may be NULL) = mean milliseconds per call
 * of the chosen configuration. */
gpm_status gpm_batch_autotune(const gpm_graph *g, const int32_t *d_voff, int32_t G, int32_t k,
                              void *d_ws, uint64_t ws_bytes, uint64_t *d_counts, void *stream,
                              int32_t reps, gpm_batch_config *best, float *best_ms);

/* ---------------------------------------------------------- serving --- */

/* A request-serving runtime (not part of the paper's method; it serves the
 * counting entry points above): requests arrive at any time; a scheduler
 * thread admits them, first come first served, whenever a slot (one HIP
 * stream each) is free and the request's workspace fits in the free part of
 * a caller-owned device memory pool; admitted requests run concurrently on
 * their slots' streams; completions are collected without blocking.  Every
 * request recomputes its answer from the resident graph. */
typedef struct gpm_server gpm_server;

typedef struct gpm_server_config {
    int32_t max_slots;      /* concurrent requests on the device, 1..64 */
    int32_t cu_percent;     /* share of the compute units one request's persistent
                               kernels are sized for, 1..100 (0: 50), so that
                               concurrent requests run side by side */
    void *d_pool;           /* device memory for request workspaces (caller-owned) */
    uint64_t pool_bytes;
} gpm_server_config;

#define GPM_QUERY_CLIQUE 1  /* k-clique count, k = 3..9 (triangles: k = 3) */
#define GPM_QUERY_MOTIF  2  /* induced k-motif counts, k = 3 or 4 */

typedef struct gpm_request {
    int32_t kind;           /* GPM_QUERY_* */
    int32_t k;
    const gpm_graph *graph; /* resident graph; must outlive the request */
    uint64_t tag;           /* caller's label, returned with the response */
} gpm_request;

typedef struct gpm_response {
    uint64_t id;            /* from gpm_server_submit */
    uint64_t tag;
    int32_t status;         /* GPM_OK or the failing status */
    int32_t n_values;       /* 1 (clique) or 2 / 6 (motif) */
    uint64_t values[7];     /* counts (motif: plus the status word) */
    double t_submit, t_admit, t_done;   /* seconds on gpm_server_now()'s clock */
    /* device clock: seconds from an event the server records at creation to
     * events recorded on the slot's stream just before and just after the
     * request's work (so d_end - d_start bounds its kernels' span on the
     * device); -1 if the device times could not be read */
    double d_start, d_end;
} gpm_response;

/* Creates the server and its scheduler thread.  Streams (default priority)
 * and a small pinned host buffer are created here; request workspaces come
 * only from the pool. */
gpm_status gpm_server_create(const gpm_server_config *cfg, gpm_server **out);
/* Queues a request (thread-safe, non-blocking); *id identifies it.  A
 * request whose workspace can never fit in the pool fails at once. */
gpm_status gpm_server_submit(gpm_server *s, const gpm_request *r, uint64_t *id);
/* Moves up to max finished responses to out; *n gets their number. */
gpm_status gpm_server_poll(gpm_server *s, gpm_response *out, int32_t max, int32_t *n);
/* Number of requests queued or running. */
int64_t gpm_server_pending(gpm_server *s);
/* Monotonic clock (seconds) used for the response timestamps. */
double gpm_server_now(void);
/* Waits for every submitted request, stops the thread, frees host state.
 * Unpolled responses are discarded. */
void gpm_server_destroy(gpm_server *s);

/* ----------------------------------------------------------- timing --- */

/* Kernel timing for measurement (off by default).  While on, the library
 * brackets each of its main kernels with HIP events recorded on the launch
 * stream.  Switch it off for production and for graph capture. */
gpm_status gpm_timing_enable(int32_t on);
/* Waits for the recorded events, writes up to cap (name, milliseconds, work
 * units) triples in launch order (names stay valid until the next call;
 * units is 0 for kernels that report none, and any pointer may be NULL),
 * clears the record, and returns the number of spans recorded (may exceed
 * cap).  Work units, where reported, are counted on the device:
 * k_tc_flat* = (v, w) pairs tested, k_lg5* = local triangles expanded. */
int32_t gpm_timing_read(const char **names, float *ms, uint64_t *units, int32_t cap);

#ifdef __cplusplus
}
#endif

#endif /* GPM_H */
