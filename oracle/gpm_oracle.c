/*
 * Plain CPU oracle for graph pattern mining counts and listings.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code with
 * the device path: its own orientation (core order), its own intersection
 * loops, its own counting formulas, its own listing hash.
 *
 * Every function takes a canonical symmetric CSR (rows sorted ascending, no
 * self-loops, no repeated neighbours, u in N(v) iff v in N(u)) with int64 row
 * offsets and int32 column ids, as built by oracle/csr.py from a raw edge
 * stream.  Counts are accumulated in unsigned 128-bit integers and returned
 * as (low, high) 64-bit halves so the caller can check their range.
 *
 * Definitions followed (Section 2, problem definition; Appendix B.7):
 *   - k-clique: a k-vertex set whose pairs are all adjacent; triangles are
 *     3-cliques.  Each vertex set counts once.
 *   - edge-induced subgraph listing: every distinct edge set F whose
 *     edge-induced subgraph is isomorphic to the pattern.
 *   - k-motifs: k-vertex sets classified by the isomorphism class of their
 *     induced subgraph; connected classes only.
 *
 * Orientation used here: degeneracy (core) order from bucket peeling, the
 * core-value alternative of Appendix B.2.  Counting each clique from its
 * first vertex in ANY total order counts it exactly once, so the order is a
 * free choice; it is deliberately not the device path's degree order.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef unsigned __int128 u128;

#define ORC_OK 0
#define ORC_BAD_ARG 1
#define ORC_NO_MEMORY 2

/* ----------------------------------------------------------- helpers --- */

static void put128(uint64_t *out, u128 x)
{
    out[0] = (uint64_t)x;
    out[1] = (uint64_t)(x >> 64);
}

/* Listing checksum = sum over embeddings of a per-embedding hash, mod 2^64.
 * Per embedding, over its canonical key sequence c_0..c_{L-1}:
 *   h = L;  then h = f((h XOR c_i) + 0x9E3779B97F4A7C15) for each i,
 * with f the splitmix64 finaliser (xor-shift 30, multiply 0xBF58476D1CE4E5B9,
 * xor-shift 27, multiply 0x94D049BB133111EB, xor-shift 31).  The key is the
 * ascending vertex tuple for vertex-induced patterns, and the ascending list
 * of edge codes (min << 32 | max) for edge-induced patterns. */
static uint64_t fin64(uint64_t z)
{
    z ^= z >> 30; z *= 0xBF58476D1CE4E5B9ULL;
    z ^= z >> 27; z *= 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return z;
}

static uint64_t key_hash(const uint64_t *key, int len)
{
    uint64_t h = (uint64_t)len;
    for (int i = 0; i < len; i++) h = fin64((h ^ key[i]) + 0x9E3779B97F4A7C15ULL);
    return h;
}

static void sort_u64(uint64_t *a, int len)
{
    for (int i = 1; i < len; i++) {           /* insertion sort; len is tiny */
        uint64_t x = a[i];
        int j = i - 1;
        while (j >= 0 && a[j] > x) { a[j + 1] = a[j]; j--; }
        a[j + 1] = x;
    }
}

static uint64_t edge_code(int32_t a, int32_t b)
{
    uint64_t lo = (uint64_t)(uint32_t)(a < b ? a : b);
    uint64_t hi = (uint64_t)(uint32_t)(a < b ? b : a);
    return (lo << 32) | hi;
}

/* |A ∩ B| for ascending arrays: two-pointer merge. */
static int64_t merge_count(const int32_t *a, int64_t na, const int32_t *b, int64_t nb)
{
    int64_t i = 0, j = 0, c = 0;
    while (i < na && j < nb) {
        if (a[i] < b[j]) i++;
        else if (a[i] > b[j]) j++;
        else { c++; i++; j++; }
    }
    return c;
}

/* A ∩ B written ascending to out; returns its size. */
static int64_t merge_into(const int32_t *a, int64_t na, const int32_t *b, int64_t nb,
                          int32_t *out)
{
    int64_t i = 0, j = 0, c = 0;
    while (i < na && j < nb) {
        if (a[i] < b[j]) i++;
        else if (a[i] > b[j]) j++;
        else { out[c++] = a[i]; i++; j++; }
    }
    return c;
}

/* ------------------------------------------------- core order + DAG --- */

/* Degeneracy order (Batagelj and Zaversnik bucket peeling): vertices are
 * removed one at a time, always one of least remaining degree; pos[v] is
 * v's removal step, a total order on the vertices. */
static int core_peel(int32_t n, const int64_t *off, const int32_t *adj, int32_t *pos,
                     int32_t *core);

static int core_positions(int32_t n, const int64_t *off, const int32_t *adj, int32_t *pos)
{
    return core_peel(n, off, adj, pos, NULL);
}

/* Core numbers (Appendix B.2's core values): a vertex's remaining degree
 * when the peeling removes it is the largest k whose k-core holds it. */
int orc_core_numbers(int32_t n, const int64_t *off, const int32_t *adj, int32_t *core)
{
    int32_t *pos = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!pos) return ORC_NO_MEMORY;
    int rc = core_peel(n, off, adj, pos, core);
    free(pos);
    return rc;
}

static int core_peel(int32_t n, const int64_t *off, const int32_t *adj, int32_t *pos,
                     int32_t *core)
{
    size_t nn = (size_t)(n > 0 ? n : 1);
    int32_t *d = malloc(sizeof(int32_t) * nn);
    int32_t *vert = malloc(sizeof(int32_t) * nn);
    int32_t *where = malloc(sizeof(int32_t) * nn);
    int32_t maxd = 0;
    if (!d || !vert || !where) { free(d); free(vert); free(where); return ORC_NO_MEMORY; }
    for (int32_t v = 0; v < n; v++) {
        d[v] = (int32_t)(off[v + 1] - off[v]);
        if (d[v] > maxd) maxd = d[v];
    }
    int32_t *bin = calloc((size_t)maxd + 2, sizeof(int32_t));
    if (!bin) { free(d); free(vert); free(where); return ORC_NO_MEMORY; }
    for (int32_t v = 0; v < n; v++) bin[d[v]]++;
    int32_t start = 0;                         /* bin[x] = first slot of degree x */
    for (int32_t x = 0; x <= maxd; x++) { int32_t c = bin[x]; bin[x] = start; start += c; }
    for (int32_t v = 0; v < n; v++) { where[v] = bin[d[v]]++; vert[where[v]] = v; }
    for (int32_t x = maxd; x >= 1; x--) bin[x] = bin[x - 1];
    bin[0] = 0;
    for (int32_t i = 0; i < n; i++) {
        int32_t v = vert[i];
        pos[v] = i;
        if (core) core[v] = d[v];
        for (int64_t e = off[v]; e < off[v + 1]; e++) {
            int32_t u = adj[e];
            if (d[u] > d[v]) {                  /* u not yet removed: lower its degree */
                int32_t du = d[u], pu = where[u], pw = bin[du], w = vert[pw];
                if (u != w) { vert[pu] = w; where[w] = pu; vert[pw] = u; where[u] = pw; }
                bin[du]++;
                d[u]--;
            }
        }
    }
    free(d); free(vert); free(where); free(bin);
    return ORC_OK;
}

/* Out-lists under the core order: N+(v) = {u in N(v) : pos[u] > pos[v]},
 * kept in ascending id order. */
static int core_dag(int32_t n, const int64_t *off, const int32_t *adj,
                    int64_t **pout, int32_t **padj, int32_t *maxout)
{
    int32_t *pos = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!pos) return ORC_NO_MEMORY;
    int rc = core_positions(n, off, adj, pos);
    if (rc) { free(pos); return rc; }
    int64_t *o = malloc(sizeof(int64_t) * ((size_t)n + 1));
    int32_t *a = malloc(sizeof(int32_t) * (size_t)(off[n] / 2 + 1));
    if (!o || !a) { free(pos); free(o); free(a); return ORC_NO_MEMORY; }
    int64_t c = 0;
    int32_t mo = 0;
    for (int32_t v = 0; v < n; v++) {
        o[v] = c;
        for (int64_t e = off[v]; e < off[v + 1]; e++)
            if (pos[adj[e]] > pos[v]) a[c++] = adj[e];
        if (c - o[v] > mo) mo = (int32_t)(c - o[v]);
    }
    o[n] = c;
    free(pos);
    *pout = o; *padj = a; *maxout = mo;
    return ORC_OK;
}

/* --------------------------------------------------------- k-cliques --- */

/* Number of cliques that extend the current prefix by `left` more vertices,
 * all drawn from cand (the common out-neighbours of the prefix). */
static u128 clique_extend(const int64_t *o, const int32_t *a, const int32_t *cand,
                          int64_t nc, int left, int32_t *scratch)
{
    if (left == 1) return (u128)nc;
    u128 total = 0;
    for (int64_t i = 0; i < nc; i++) {
        int32_t w = cand[i];
        int64_t nn = merge_into(cand, nc, a + o[w], o[w + 1] - o[w], scratch);
        if (nn >= left - 1) total += clique_extend(o, a, scratch, nn, left - 1, scratch + nn);
    }
    return total;
}

/* Number of k-vertex cliques, k >= 1. */
int orc_clique_count(int32_t n, const int64_t *off, const int32_t *adj, int32_t k,
                     int32_t threads, uint64_t *out)
{
    if (n < 0 || k < 1 || !out) return ORC_BAD_ARG;
    if (k == 1) { put128(out, (u128)(uint64_t)n); return ORC_OK; }
    if (k == 2) { put128(out, (u128)(uint64_t)(off[n] / 2)); return ORC_OK; }
    int64_t *o; int32_t *a; int32_t mo;
    int rc = core_dag(n, off, adj, &o, &a, &mo);
    if (rc) return rc;
    u128 total = 0;
    int failed = 0;
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel reduction(+ : total) reduction(| : failed)
    {
        int32_t *scratch = malloc(sizeof(int32_t) * ((size_t)mo * (size_t)k + 1));
        if (!scratch) failed = 1;
#pragma omp for schedule(dynamic, 64)
        for (int32_t v = 0; v < n; v++) {
            if (!scratch) continue;
            int64_t d = o[v + 1] - o[v];
            if (d >= k - 1) total += clique_extend(o, a, a + o[v], d, k - 1, scratch);
        }
        free(scratch);
    }
    free(o); free(a);
    if (failed) return ORC_NO_MEMORY;
    put128(out, total);
    return ORC_OK;
}

/* The core-ordered DAG built once, for counting cliques rooted at chosen
 * vertices (a share of the roots) without rebuilding it per call.  pos is
 * each vertex's position in the core order, o / a the out-lists. */
struct orc_dag {
    int32_t n, maxout;
    int32_t *pos;
    int64_t *o;
    int32_t *a;
};

int orc_dag_build(int32_t n, const int64_t *off, const int32_t *adj, struct orc_dag **out)
{
    if (n < 0 || !out) return ORC_BAD_ARG;
    struct orc_dag *g = calloc(1, sizeof(*g));
    if (!g) return ORC_NO_MEMORY;
    g->n = n;
    g->pos = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!g->pos) { free(g); return ORC_NO_MEMORY; }
    int rc = core_positions(n, off, adj, g->pos);
    if (!rc) rc = core_dag(n, off, adj, &g->o, &g->a, &g->maxout);
    if (rc) { free(g->pos); free(g); return rc; }
    *out = g;
    return ORC_OK;
}

void orc_dag_free(struct orc_dag *g)
{
    if (!g) return;
    free(g->pos); free(g->o); free(g->a); free(g);
}

/* Number of k-cliques (k >= 3) whose first vertex in the core order has a
 * position p with p % stride == offset.  Every clique has exactly one first
 * vertex, so the counts over offsets 0..stride-1 add up to orc_clique_count,
 * and stride 1 is orc_clique_count itself.  Used to time the oracle on a
 * bounded share of a workload's roots. */
int orc_dag_clique_count_sampled(const struct orc_dag *g, int32_t k, int32_t threads,
                                 int32_t stride, int32_t offset, uint64_t *out)
{
    if (!g || k < 3 || stride < 1 || offset < 0 || offset >= stride || !out) return ORC_BAD_ARG;
    const int64_t *o = g->o;
    const int32_t *a = g->a, *pos = g->pos;
    u128 total = 0;
    int failed = 0;
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel reduction(+ : total) reduction(| : failed)
    {
        int32_t *scratch = malloc(sizeof(int32_t) * ((size_t)g->maxout * (size_t)k + 1));
        if (!scratch) failed = 1;
#pragma omp for schedule(dynamic, 64)
        for (int32_t v = 0; v < g->n; v++) {
            if (!scratch || pos[v] % stride != offset) continue;
            int64_t d = o[v + 1] - o[v];
            if (d >= k - 1) total += clique_extend(o, a, a + o[v], d, k - 1, scratch);
        }
        free(scratch);
    }
    if (failed) return ORC_NO_MEMORY;
    put128(out, total);
    return ORC_OK;
}

/* The same share, building (and freeing) the core-ordered DAG in the call. */
int orc_clique_count_sampled(int32_t n, const int64_t *off, const int32_t *adj, int32_t k,
                             int32_t threads, int32_t stride, int32_t offset, uint64_t *out)
{
    if (n < 0 || k < 3 || stride < 1 || offset < 0 || offset >= stride || !out)
        return ORC_BAD_ARG;
    struct orc_dag *g;
    int rc = orc_dag_build(n, off, adj, &g);
    if (rc) return rc;
    rc = orc_dag_clique_count_sampled(g, k, threads, stride, offset, out);
    orc_dag_free(g);
    return rc;
}

/* Lists every k-clique (k >= 3) as its ascending vertex tuple.  The first
 * `cap` found are written to buf (k ints each, in an unspecified order);
 * total and the checksum cover all of them. */
struct list_sink {
    int32_t *buf;
    uint64_t cap;
    uint64_t written;   /* shared slot counter (atomic) */
};

static void sink_emit(struct list_sink *s, const int32_t *tuple, int k)
{
    uint64_t slot, seen;
    /* once the buffer is full, stop touching the shared counter */
#pragma omp atomic read
    seen = s->written;
    if (seen >= s->cap) return;
#pragma omp atomic capture
    slot = s->written++;
    if (slot < s->cap) memcpy(s->buf + slot * (uint64_t)k, tuple, sizeof(int32_t) * (size_t)k);
}

static void clique_list_rec(const int64_t *o, const int32_t *a, const int32_t *cand, int64_t nc,
                            int depth, int k, int32_t *prefix, int32_t *scratch,
                            struct list_sink *s, uint64_t *cnt, uint64_t *sum)
{
    for (int64_t i = 0; i < nc; i++) {
        prefix[depth] = cand[i];
        if (depth == k - 1) {
            uint64_t key[16];
            for (int t = 0; t < k; t++) key[t] = (uint64_t)(uint32_t)prefix[t];
            sort_u64(key, k);
            *sum += key_hash(key, k);
            (*cnt)++;
            sink_emit(s, prefix, k);
        } else {
            int32_t w = cand[i];
            int64_t nn = merge_into(cand, nc, a + o[w], o[w + 1] - o[w], scratch);
            clique_list_rec(o, a, scratch, nn, depth + 1, k, prefix, scratch + nn, s, cnt, sum);
        }
    }
}

int orc_clique_list(int32_t n, const int64_t *off, const int32_t *adj, int32_t k,
                    int32_t threads, int32_t *buf, uint64_t cap,
                    uint64_t *total, uint64_t *written, uint64_t *checksum)
{
    if (n < 0 || k < 3 || k > 16 || !total || !written || !checksum) return ORC_BAD_ARG;
    int64_t *o; int32_t *a; int32_t mo;
    int rc = core_dag(n, off, adj, &o, &a, &mo);
    if (rc) return rc;
    struct list_sink s = { buf, buf ? cap : 0, 0 };
    uint64_t cnt = 0, sum = 0;
    int failed = 0;
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel reduction(+ : cnt, sum) reduction(| : failed)
    {
        int32_t *scratch = malloc(sizeof(int32_t) * ((size_t)mo * (size_t)k + 1));
        int32_t prefix[16];
        if (!scratch) failed = 1;
#pragma omp for schedule(dynamic, 64)
        for (int32_t v = 0; v < n; v++) {
            if (!scratch) continue;
            prefix[0] = v;
            clique_list_rec(o, a, a + o[v], o[v + 1] - o[v], 1, k, prefix, scratch, &s, &cnt, &sum);
        }
        free(scratch);
    }
    free(o); free(a);
    if (failed) return ORC_NO_MEMORY;
    *total = cnt;
    *written = cnt < s.cap ? cnt : s.cap;
    *checksum = sum;
    return ORC_OK;
}

/* ------------------------------------------ per-edge triangle counts --- */

/* te[e] = |N(x) ∩ N(y)| for every arc e = (x, y) of the symmetric CSR. */
int orc_edge_triangles(int32_t n, const int64_t *off, const int32_t *adj, int32_t threads,
                       int64_t *te)
{
    if (n < 0 || !te) return ORC_BAD_ARG;
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel for schedule(dynamic, 64)
    for (int32_t x = 0; x < n; x++)
        for (int64_t e = off[x]; e < off[x + 1]; e++) {
            int32_t y = adj[e];
            te[e] = merge_count(adj + off[x], off[x + 1] - off[x], adj + off[y], off[y + 1] - off[y]);
        }
    return ORC_OK;
}

/* ------------------------------ non-induced 4-vertex subgraph counts --- */

/* Sum over unordered vertex pairs {x, z} of C(codeg(x, z), 2), where codeg
 * is the number of common neighbours.  Each 4-cycle has two diagonals, so
 * this sum is twice the number of (not necessarily induced) 4-cycles. */
static int pair_codegree_sum(int32_t n, const int64_t *off, const int32_t *adj, u128 *res)
{
    u128 total = 0;
    int failed = 0;
#pragma omp parallel reduction(+ : total) reduction(| : failed)
    {
        int32_t *cnt = calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
        int32_t *touched = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
        if (!cnt || !touched) failed = 1;
#pragma omp for schedule(dynamic, 16)
        for (int32_t x = 0; x < n; x++) {
            if (failed) continue;
            int32_t nt = 0;
            for (int64_t e = off[x]; e < off[x + 1]; e++) {
                int32_t y = adj[e];
                for (int64_t f = off[y]; f < off[y + 1]; f++) {
                    int32_t z = adj[f];
                    if (z <= x) continue;        /* unordered pair {x, z}, x < z */
                    if (cnt[z]++ == 0) touched[nt++] = z;
                }
            }
            for (int32_t t = 0; t < nt; t++) {
                uint64_t c = (uint64_t)cnt[touched[t]];
                total += (u128)(c * (c - 1) / 2);
                cnt[touched[t]] = 0;
            }
        }
        free(cnt); free(touched);
    }
    if (failed) return ORC_NO_MEMORY;
    *res = total;
    return ORC_OK;
}

/* Counts of subgraphs (not necessarily induced) on 4 vertices, as 128-bit
 * pairs in out[12], in the order
 *   claw (3-star), 4-path, 4-cycle, paw (tailed triangle), diamond, 4-clique.
 * Closed forms, each counting every copy once:
 *   claw    = sum_v C(d_v, 3)                       (centre, 3 leaves)
 *   4-path  = sum_{xy in E} (d_x - 1)(d_y - 1) - 3T (middle edge, two ends;
 *             the ends coincide exactly on the 3 edges of each triangle)
 *   4-cycle = (1/2) sum_{x<z} C(codeg(x,z), 2)
 *   paw     = sum_v t_v (d_v - 2)                   (triangle at v, tail at v)
 *   diamond = sum_{xy in E} C(T_xy, 2)              (the diagonal xy)
 *   4-clique from the clique counter. */
int orc_motif4_noninduced(int32_t n, const int64_t *off, const int32_t *adj, int32_t threads,
                          uint64_t *out)
{
    if (n < 0 || !out) return ORC_BAD_ARG;
    if (threads > 0) omp_set_num_threads(threads);
    int64_t arcs = off[n];
    int64_t *te = malloc(sizeof(int64_t) * (size_t)(arcs > 0 ? arcs : 1));
    if (!te) return ORC_NO_MEMORY;
    int rc = orc_edge_triangles(n, off, adj, threads, te);
    if (rc) { free(te); return rc; }
    u128 claw = 0, p4a = 0, paw = 0, dia = 0, tri3 = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : claw, p4a, paw, dia, tri3)
    for (int32_t x = 0; x < n; x++) {
        uint64_t dx = (uint64_t)(off[x + 1] - off[x]);
        if (dx >= 3) claw += (u128)dx * (dx - 1) * (dx - 2) / 6;
        uint64_t tx2 = 0;                      /* 2 t_x = sum over arcs at x of T */
        for (int64_t e = off[x]; e < off[x + 1]; e++) {
            int32_t y = adj[e];
            uint64_t dy = (uint64_t)(off[y + 1] - off[y]);
            uint64_t t = (uint64_t)te[e];
            tx2 += t;
            if (y > x) {                       /* each undirected edge once */
                p4a += (u128)(dx - 1) * (dy - 1);
                if (t >= 2) dia += (u128)t * (t - 1) / 2;
                tri3 += t;                     /* sum_e T_e = 3T */
            }
        }
        if (dx >= 2) paw += (u128)(tx2 / 2) * (dx - 2);
    }
    free(te);
    u128 c4x2;
    rc = pair_codegree_sum(n, off, adj, &c4x2);
    if (rc) return rc;
    uint64_t k4[2];
    rc = orc_clique_count(n, off, adj, 4, threads, k4);
    if (rc) return rc;
    put128(out + 0, claw);
    put128(out + 2, p4a - tri3);               /* tri3 = 3T */
    put128(out + 4, c4x2 / 2);
    put128(out + 6, paw);
    put128(out + 8, dia);
    out[10] = k4[0]; out[11] = k4[1];
    return ORC_OK;
}

/* --------------------------------------- edge-induced listing (SL) --- */

/* Edge-induced diamonds.  A diamond's diagonal is its only edge whose two
 * ends both have degree 3 inside it, so each diamond is found exactly once
 * as (diagonal a<b, tips c<d with c, d in N(a) ∩ N(b)); its edge set is
 * {ab, ac, ad, bc, bd}.  Written as (a, b, c, d). */
int orc_list_diamonds(int32_t n, const int64_t *off, const int32_t *adj, int32_t threads,
                      int32_t *buf, uint64_t cap, uint64_t *total, uint64_t *written,
                      uint64_t *checksum)
{
    if (n < 0 || !total || !written || !checksum) return ORC_BAD_ARG;
    int32_t maxd = 0;
    for (int32_t v = 0; v < n; v++)
        if (off[v + 1] - off[v] > maxd) maxd = (int32_t)(off[v + 1] - off[v]);
    struct list_sink s = { buf, buf ? cap : 0, 0 };
    uint64_t cnt = 0, sum = 0;
    int failed = 0;
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel reduction(+ : cnt, sum) reduction(| : failed)
    {
        int32_t *common = malloc(sizeof(int32_t) * ((size_t)maxd + 1));
        if (!common) failed = 1;
#pragma omp for schedule(dynamic, 64)
        for (int32_t a = 0; a < n; a++) {
            if (!common) continue;
            for (int64_t e = off[a]; e < off[a + 1]; e++) {
                int32_t b = adj[e];
                if (b <= a) continue;
                int64_t t = merge_into(adj + off[a], off[a + 1] - off[a],
                                       adj + off[b], off[b + 1] - off[b], common);
                for (int64_t i = 0; i < t; i++)
                    for (int64_t j = i + 1; j < t; j++) {
                        int32_t c = common[i], d = common[j];
                        uint64_t key[5] = { edge_code(a, b), edge_code(a, c), edge_code(a, d),
                                            edge_code(b, c), edge_code(b, d) };
                        sort_u64(key, 5);
                        sum += key_hash(key, 5);
                        cnt++;
                        int32_t tup[4] = { a, b, c, d };
                        sink_emit(&s, tup, 4);
                    }
            }
        }
        free(common);
    }
    if (failed) return ORC_NO_MEMORY;
    *total = cnt;
    *written = cnt < s.cap ? cnt : s.cap;
    *checksum = sum;
    return ORC_OK;
}

/* Edge-induced 4-cycles v0-v1-v2-v3-v0.  Each cycle is found once from its
 * smallest vertex v0, opposite vertex v2, and the pair v1 < v3 of v0's
 * neighbours adjacent to v2.  Written as (v0, v1, v2, v3). */
int orc_list_c4(int32_t n, const int64_t *off, const int32_t *adj, int32_t threads,
                int32_t *buf, uint64_t cap, uint64_t *total, uint64_t *written,
                uint64_t *checksum)
{
    if (n < 0 || !total || !written || !checksum) return ORC_BAD_ARG;
    struct list_sink s = { buf, buf ? cap : 0, 0 };
    uint64_t cnt = 0, sum = 0;
    int failed = 0;
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel reduction(+ : cnt, sum) reduction(| : failed)
    {
        size_t nn = (size_t)(n > 0 ? n : 1);
        int32_t *head = malloc(sizeof(int32_t) * nn);   /* per v2: chain of middles */
        int32_t *touched = malloc(sizeof(int32_t) * nn);
        int64_t nodes_cap = 1024;
        int32_t *node_mid = malloc(sizeof(int32_t) * (size_t)nodes_cap);
        int32_t *node_next = malloc(sizeof(int32_t) * (size_t)nodes_cap);
        int32_t *mids = malloc(sizeof(int32_t) * nn);
        if (!head || !touched || !node_mid || !node_next || !mids) failed = 1;
        else for (size_t i = 0; i < nn; i++) head[i] = -1;
#pragma omp for schedule(dynamic, 16)
        for (int32_t v0 = 0; v0 < n; v0++) {
            if (failed) continue;
            int32_t nt = 0;
            int64_t nodes = 0;
            for (int64_t e = off[v0]; e < off[v0 + 1]; e++) {
                int32_t v1 = adj[e];
                if (v1 <= v0) continue;
                for (int64_t f = off[v1]; f < off[v1 + 1]; f++) {
                    int32_t v2 = adj[f];
                    if (v2 <= v0) continue;
                    if (nodes == nodes_cap) {
                        nodes_cap *= 2;
                        int32_t *a1 = realloc(node_mid, sizeof(int32_t) * (size_t)nodes_cap);
                        int32_t *a2 = realloc(node_next, sizeof(int32_t) * (size_t)nodes_cap);
                        if (a1) node_mid = a1;
                        if (a2) node_next = a2;
                        if (!a1 || !a2) { failed = 1; break; }
                    }
                    if (head[v2] < 0) touched[nt++] = v2;
                    node_mid[nodes] = v1;
                    node_next[nodes] = head[v2];
                    head[v2] = (int32_t)nodes;
                    nodes++;
                }
                if (failed) break;
            }
            for (int32_t t = 0; t < nt; t++) {
                int32_t v2 = touched[t];
                int32_t nm = 0;
                for (int32_t p = head[v2]; p >= 0; p = node_next[p]) mids[nm++] = node_mid[p];
                head[v2] = -1;
                for (int32_t i = 0; i < nm; i++)
                    for (int32_t j = i + 1; j < nm; j++) {
                        int32_t v1 = mids[i] < mids[j] ? mids[i] : mids[j];
                        int32_t v3 = mids[i] < mids[j] ? mids[j] : mids[i];
                        uint64_t key[4] = { edge_code(v0, v1), edge_code(v1, v2),
                                            edge_code(v2, v3), edge_code(v3, v0) };
                        sort_u64(key, 4);
                        sum += key_hash(key, 4);
                        cnt++;
                        int32_t tup[4] = { v0, v1, v2, v3 };
                        sink_emit(&s, tup, 4);
                    }
            }
        }
        free(head); free(touched); free(node_mid); free(node_next); free(mids);
    }
    if (failed) return ORC_NO_MEMORY;
    *total = cnt;
    *written = cnt < s.cap ? cnt : s.cap;
    *checksum = sum;
    return ORC_OK;
}

/* Degree statistics used by measurement: sum_v C(d_v, 2) (wedges centred
 * anywhere), as a 128-bit pair. */
int orc_wedges(int32_t n, const int64_t *off, uint64_t *out)
{
    if (n < 0 || !out) return ORC_BAD_ARG;
    u128 w = 0;
    for (int32_t v = 0; v < n; v++) {
        uint64_t d = (uint64_t)(off[v + 1] - off[v]);
        if (d >= 2) w += (u128)d * (d - 1) / 2;
    }
    put128(out, w);
    return ORC_OK;
}

/* ------------------------------------------------ any connected pattern --- */
/*
 * Embeddings of a connected pattern P (k <= 8 vertices, edge list pe[2*ne])
 * in G (Section 2: subgraph listing counts edge-induced embeddings, motif
 * counting vertex-induced ones).  Written as the plain definition: count
 * every injective map f from P's vertices to G's with f(a)f(b) an edge of G
 * for each pattern edge ab (and, vertex-induced, a non-edge for each pattern
 * non-edge), then divide by |Aut(P)|, the number of such maps per
 * embedding.  No symmetry breaking.  Pattern vertices are visited in BFS
 * order from vertex 0 so each one after the first has an earlier neighbour
 * whose row supplies its candidates.
 */
static int has_edge(const int64_t *off, const int32_t *adj, int32_t u, int32_t v)
{
    int64_t lo = off[u], hi = off[u + 1];
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (adj[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo < off[u + 1] && adj[lo] == v;
}

struct pat {
    int k, induced;
    int order[8];          /* pattern vertex visited at step i */
    int adjm[8][8];        /* pattern adjacency by vertex */
    int anchor[8];         /* an earlier step adjacent to step i */
};

static u128 maps_from(const int64_t *off, const int32_t *adj, const struct pat *p,
                      int32_t *img, int step)
{
    if (step == p->k) return 1;
    const int pv = p->order[step];
    const int32_t a = img[p->anchor[step]];
    u128 total = 0;
    for (int64_t e = off[a]; e < off[a + 1]; e++) {
        const int32_t v = adj[e];
        int ok = 1;
        for (int s = 0; s < step && ok; s++) {
            if (img[s] == v) { ok = 0; break; }
            const int adjacent = p->adjm[pv][p->order[s]];
            if (s == p->anchor[step]) continue;
            const int edge = has_edge(off, adj, img[s], v);
            if (adjacent && !edge) ok = 0;
            if (!adjacent && p->induced && edge) ok = 0;
        }
        if (!ok) continue;
        img[step] = v;
        total += maps_from(off, adj, p, img, step + 1);
    }
    return total;
}

static int next_perm(int *a, int n)
{
    int i = n - 2;
    while (i >= 0 && a[i] >= a[i + 1]) i--;
    if (i < 0) return 0;
    int j = n - 1;
    while (a[j] <= a[i]) j--;
    int t = a[i]; a[i] = a[j]; a[j] = t;
    for (int l = i + 1, r = n - 1; l < r; l++, r--) { t = a[l]; a[l] = a[r]; a[r] = t; }
    return 1;
}

/* out[0..1]: embeddings (low, high); out[2]: |Aut(P)|. */
int orc_pattern_count(int32_t n, const int64_t *off, const int32_t *adj, int32_t k, int32_t ne,
                      const int32_t *pe, int32_t induced, int32_t threads, uint64_t *out)
{
    if (n < 0 || k < 2 || k > 8 || ne < k - 1 || !pe || !out) return ORC_BAD_ARG;
    struct pat p;
    memset(&p, 0, sizeof(p));
    p.k = k;
    p.induced = induced != 0;
    for (int i = 0; i < ne; i++) {
        const int a = pe[2 * i], b = pe[2 * i + 1];
        if (a < 0 || b < 0 || a >= k || b >= k || a == b) return ORC_BAD_ARG;
        p.adjm[a][b] = p.adjm[b][a] = 1;
    }
    /* BFS order from vertex 0; the anchor of each step is its BFS parent */
    int seen[8] = {0}, parent_step[8] = {0}, head = 0, tail = 0;
    p.order[tail++] = 0;
    seen[0] = 1;
    while (head < tail) {
        const int x = p.order[head];
        for (int y = 0; y < k; y++)
            if (p.adjm[x][y] && !seen[y]) {
                seen[y] = 1;
                parent_step[tail] = head;
                p.order[tail++] = y;
            }
        head++;
    }
    if (tail != k) return ORC_BAD_ARG;   /* not connected */
    for (int i = 1; i < k; i++) p.anchor[i] = parent_step[i];
    /* |Aut(P)|: permutations preserving adjacency */
    int perm[8];
    for (int i = 0; i < k; i++) perm[i] = i;
    uint64_t aut = 0;
    do {
        int ok = 1;
        for (int a = 0; a < k && ok; a++)
            for (int b = 0; b < k; b++)
                if (p.adjm[a][b] != p.adjm[perm[a]][perm[b]]) { ok = 0; break; }
        aut += ok;
    } while (next_perm(perm, k));
    u128 total = 0;
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : total)
    for (int32_t r = 0; r < n; r++) {
        int32_t img[8];
        img[0] = r;
        total += maps_from(off, adj, &p, img, 1);
    }
    if (total % aut != 0) return ORC_BAD_ARG;   /* cannot happen for a valid pattern */
    put128(out, total / aut);
    out[2] = aut;
    return ORC_OK;
}


/* Listing of a connected pattern's embeddings (Section 2, subgraph listing;
 * vertex- or edge-induced as in orc_pattern_count).  Each embedding is
 * reported once: among the |Aut(P)| injective maps that give it, the one
 * whose image vector (f(0), ..., f(k-1)) is lexicographically smallest.
 * Rows hold f(0..k-1); the checksum term uses the key of the comment above
 * (vertex tuple or edge codes, ascending). */
struct plist {
    const struct pat *p;
    int ne;
    int pe[28][2];
    int naut;
    int *aut;              /* naut maps of k entries */
    struct list_sink sink;
    uint64_t total, sum;
};

static void plist_found(struct plist *L, const int32_t *img)
{
    const struct pat *p = L->p;
    const int k = p->k;
    int32_t f[8];
    for (int s = 0; s < k; s++) f[p->order[s]] = img[s];
    for (int t = 0; t < L->naut; t++) {
        const int *sg = L->aut + (size_t)t * k;
        for (int x = 0; x < k; x++) {
            const int32_t g = f[sg[x]];
            if (g < f[x]) return;          /* an automorphic copy comes first */
            if (g > f[x]) break;
        }
    }
    uint64_t key[28];
    int len;
    if (p->induced) {
        for (int x = 0; x < k; x++) key[x] = (uint64_t)(uint32_t)f[x];
        len = k;
    } else {
        for (int i = 0; i < L->ne; i++) {
            const uint32_t a = (uint32_t)f[L->pe[i][0]], b = (uint32_t)f[L->pe[i][1]];
            key[i] = a < b ? ((uint64_t)a << 32) | b : ((uint64_t)b << 32) | a;
        }
        len = L->ne;
    }
    sort_u64(key, len);
    L->sum += key_hash(key, len);
    L->total++;
    sink_emit(&L->sink, f, k);
}

static void plist_from(const int64_t *off, const int32_t *adj, struct plist *L, int32_t *img,
                       int step)
{
    const struct pat *p = L->p;
    if (step == p->k) { plist_found(L, img); return; }
    const int pv = p->order[step];
    const int32_t a = img[p->anchor[step]];
    for (int64_t e = off[a]; e < off[a + 1]; e++) {
        const int32_t v = adj[e];
        int ok = 1;
        for (int s = 0; s < step && ok; s++) {
            if (img[s] == v) { ok = 0; break; }
            const int adjacent = p->adjm[pv][p->order[s]];
            if (s == p->anchor[step]) continue;
            const int edge = has_edge(off, adj, img[s], v);
            if (adjacent && !edge) ok = 0;
            if (!adjacent && p->induced && edge) ok = 0;
        }
        if (!ok) continue;
        img[step] = v;
        plist_from(off, adj, L, img, step + 1);
    }
}

int orc_pattern_list(int32_t n, const int64_t *off, const int32_t *adj, int32_t k, int32_t ne,
                     const int32_t *pe, int32_t induced, int32_t *buf, uint64_t cap,
                     uint64_t *total, uint64_t *written, uint64_t *checksum)
{
    if (n < 0 || k < 2 || k > 8 || ne < k - 1 || ne > 28 || !pe || !total || !written ||
        !checksum)
        return ORC_BAD_ARG;
    struct pat p;
    memset(&p, 0, sizeof(p));
    p.k = k;
    p.induced = induced != 0;
    struct plist L;
    memset(&L, 0, sizeof(L));
    L.p = &p;
    L.ne = ne;
    for (int i = 0; i < ne; i++) {
        const int a = pe[2 * i], b = pe[2 * i + 1];
        if (a < 0 || b < 0 || a >= k || b >= k || a == b) return ORC_BAD_ARG;
        p.adjm[a][b] = p.adjm[b][a] = 1;
        L.pe[i][0] = a;
        L.pe[i][1] = b;
    }
    int seen[8] = {0}, parent_step[8] = {0}, head = 0, tail = 0;
    p.order[tail++] = 0;
    seen[0] = 1;
    while (head < tail) {
        const int x = p.order[head];
        for (int y = 0; y < k; y++)
            if (p.adjm[x][y] && !seen[y]) {
                seen[y] = 1;
                parent_step[tail] = head;
                p.order[tail++] = y;
            }
        head++;
    }
    if (tail != k) return ORC_BAD_ARG;
    for (int i = 1; i < k; i++) p.anchor[i] = parent_step[i];
    int perm[8];
    size_t fact = 1;
    for (int i = 2; i <= k; i++) fact *= (size_t)i;
    L.aut = malloc(sizeof(int) * fact * (size_t)k);
    if (!L.aut) return ORC_NO_MEMORY;
    for (int i = 0; i < k; i++) perm[i] = i;
    do {
        int ok = 1;
        for (int a = 0; a < k && ok; a++)
            for (int b = 0; b < k; b++)
                if (p.adjm[a][b] != p.adjm[perm[a]][perm[b]]) { ok = 0; break; }
        if (ok) memcpy(L.aut + (size_t)L.naut++ * k, perm, sizeof(int) * (size_t)k);
    } while (next_perm(perm, k));
    L.sink.buf = buf;
    L.sink.cap = buf ? cap : 0;
    L.sink.written = 0;
    for (int32_t r = 0; r < n; r++) {
        int32_t img[8];
        img[0] = r;
        plist_from(off, adj, &L, img, 1);
    }
    free(L.aut);
    *total = L.total;
    *written = L.sink.written < L.sink.cap ? L.sink.written : L.sink.cap;
    *checksum = L.sum;
    return ORC_OK;
}
