/*
 * Picasso palette colouring -- plain CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * single-threaded reference that the HIP path is checked against.  It shares
 * no code, header, table or constant with the GPU library; only the tests,
 * the smoke check and the benchmark's CPU-baseline leg may load it.
 *
 * Every function follows a passage of the paper (Picasso: memory-efficient
 * graph coloring using palettes, arXiv 2401.06713) and cites it by section,
 * equation or algorithm.  Where the paper is silent the reading used here is
 * stated beside the code; the same readings are listed in the design notes.
 *
 * Pinning status (what fixes each function other than this file):
 *   relation        -- Kronecker products of the Pauli matrices, per-qubit
 *                      matrix commutators, the paper's 3-bit code, and the
 *                      Jordan-Wigner / {I,Z} special cases (tests).
 *   params          -- the list/palette sizes printed for the paper-scale
 *                      configurations (2 ln 2000 -> 16, 0.125*2000 -> 250).
 *   philox          -- the generator's published known-answer vectors
 *                      (Salmon et al., SC'11), stored as a test fixture.
 *   sampler         -- pinned by structure (T distinct sorted values in
 *                      range, T = P gives the whole palette) and by statistics
 *                      (marginals T/P, pair-share probability, bucket pairs).
 *   conflict edges  -- brute force on tiny inputs, T = P special case, the
 *                      closed-form expectation of |E_c|.
 *   greedy colouring-- validity, list respect, progress, textbook greedy when
 *                      T = P, complete and empty relation graphs, chromatic
 *                      lower bound by subset DP for n <= 12.  Exact colour
 *                      values beyond these are parity unpinned by the paper.
 *   dynamic colourer-- (Alg. 2) a pure-Python replay of its rules from the
 *                      reported order and colours, uniform first choices,
 *                      empty and complete graphs, full-run validity.
 *   schedule driver -- a constant schedule reproduces the fixed-parameter run.
 *   features        -- direct counts (weight), density 1 / 0 on complete and
 *                      empty relation graphs, closed-form density for i.i.d.
 *   predictor twin  -- gradients against central finite differences, the
 *                      forward pass against the collapsed affine map, Adam's
 *                      first step in closed form.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_REL_ANTICOMMUTE 0
#define ORC_REL_QWC 1
#define ORC_REL_COMMUTE 2

/* ------------------------------------------------------------------------ */
/* Pauli strings and the pairwise relation (Sec. IV-A, Eq. 4-5; Sec. III)     */
/* ------------------------------------------------------------------------ */

/* Qubit k of a string held as two bit-planes: (x,z) = (0,0) I, (1,0) X,
 * (1,1) Y, (0,1) Z.  Qubit k is bit k%64 of word k/64. */
static char pauli_char(const uint64_t *x, const uint64_t *z, int k)
{
    int xb = (int)((x[k / 64] >> (k % 64)) & 1u);
    int zb = (int)((z[k / 64] >> (k % 64)) & 1u);
    if (xb && zb) return 'Y';
    if (xb) return 'X';
    if (zb) return 'Z';
    return 'I';
}

/* Decode n strings of q qubits into characters, n*q bytes, row-major. */
void orc_decode(int64_t n, int32_t q, const uint64_t *x, const uint64_t *z, char *out)
{
    int W = (q + 63) / 64;
    for (int64_t i = 0; i < n; i++)
        for (int k = 0; k < q; k++)
            out[i * q + k] = pauli_char(x + i * W, z + i * W, k);
}

/* Two single-qubit Pauli matrices anticommute exactly when both are
 * non-identity and they differ (Eq. 5); every other pair commutes. */
int orc_qubit_anticommutes(char a, char b)
{
    return a != 'I' && b != 'I' && a != b;
}

/* Relation on two decoded strings.
 * ANTICOMMUTE: the strings anticommute iff the number of anticommuting
 *              positions is odd (Sec. IV-A, the parity rule after Eq. 5).
 * QWC:         "not qubit-wise commuting": some position anticommutes
 *              (qubit-wise commutativity, Sec. III).
 * COMMUTE:     the strings commute (even count): the orientation of the
 *              paper's own application (Sec. II and Sec. IV-A), whose colour
 *              classes are sets of mutually anticommuting strings.
 * Returns 1 when the pair fails the grouping relation (a graph edge). */
int orc_relation_chars(int32_t q, const char *a, const char *b, int32_t rel)
{
    int count = 0;
    for (int k = 0; k < q; k++)
        if (orc_qubit_anticommutes(a[k], b[k])) count++;
    if (rel == ORC_REL_ANTICOMMUTE) return count % 2 == 1;
    if (rel == ORC_REL_COMMUTE) return count % 2 == 0;
    return count > 0;
}

/* ------------------------------------------------------------------------ */
/* Counter-based random numbers                                              */
/* ------------------------------------------------------------------------ */

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the
 * two-multiplier Feistel-like bijection on a 4x32-bit counter, the 2x32-bit
 * key bumped by the Weyl constants between rounds. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

#define ORC_TAG_LIST 0x4C495354u /* colour-list draws */
#define ORC_TAG_PRIO 0x5052494Fu /* vertex priorities */

/* 64-bit draw keyed by (seed; vertex, slot, iteration, tag): counter
 * (v, s, ell, tag), key (seed low, seed high); the value is word1:word0. */
uint64_t orc_hash64(uint64_t seed, uint32_t v, uint32_t s, uint32_t ell, uint32_t tag)
{
    uint32_t ctr[4] = {v, s, ell, tag};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return ((uint64_t)out[1] << 32) | out[0];
}

/* ------------------------------------------------------------------------ */
/* Per-iteration palette and list size (Alg. 1 "estimate" step; Table I;      */
/* Sec. VII: P is a percentage of |V|, L = alpha log|V|, same every iteration)*/
/* Readings: natural log, ceiling, P >= 1, 1 <= T <= P.                       */
/* ------------------------------------------------------------------------ */
void orc_params(int64_t m, double frac, double alpha, int32_t fixed_T, int64_t *P_out, int32_t *T_out)
{
    double pd = ceil(frac * (double)m);
    int64_t P = (int64_t)pd;
    if (P < 1) P = 1;
    int64_t T;
    if (fixed_T > 0) {
        T = fixed_T;
    } else {
        double td = ceil(alpha * log((double)m));
        T = (int64_t)td;
    }
    if (T < 1) T = 1;
    if (T > P) T = P;
    *P_out = P;
    *T_out = (int32_t)T;
}

/* ------------------------------------------------------------------------ */
/* Random colour lists (Alg. 1 assign_rand_list_colors; Sec. IV: each vertex  */
/* gets T colours chosen uniformly at random from the palette).               */
/* Reading: a uniform T-subset drawn with Floyd's algorithm (Bentley & Floyd, */
/* CACM 1987), one keyed draw per step, then sorted ascending.                */
/* ------------------------------------------------------------------------ */
static uint64_t mul_high64(uint64_t a, uint64_t b)
{
    unsigned __int128 p = (unsigned __int128)a * b;
    return (uint64_t)(p >> 64);
}

void orc_sample_list(uint64_t seed, uint32_t ell, uint32_t v, int64_t P, int32_t T, uint32_t *out)
{
    int cnt = 0;
    for (int s = 0; s < T; s++) {
        uint64_t j = (uint64_t)(P - T + s);
        uint64_t r = orc_hash64(seed, v, (uint32_t)s, ell, ORC_TAG_LIST);
        uint64_t t = mul_high64(r, j + 1); /* uniform-ish in [0, j] */
        int present = 0;
        for (int i = 0; i < cnt; i++)
            if (out[i] == (uint32_t)t) present = 1;
        out[cnt++] = present ? (uint32_t)j : (uint32_t)t;
    }
    /* insertion sort, ascending */
    for (int i = 1; i < cnt; i++) {
        uint32_t key = out[i];
        int k = i - 1;
        while (k >= 0 && out[k] > key) {
            out[k + 1] = out[k];
            k--;
        }
        out[k + 1] = key;
    }
}

/* Vertex priority for the random static order (Sec. IV-B, static schemes,
 * "Random ordering").  Reading: u precedes v iff (prio(u), u) < (prio(v), v). */
uint64_t orc_priority(uint64_t seed, uint32_t ell, uint32_t v)
{
    return orc_hash64(seed, v, 0, ell, ORC_TAG_PRIO);
}

/* Lists of the vertices ids[0..m) (original ids), row-major m x T. */
void orc_sample_lists(uint64_t seed, uint32_t ell, int64_t m, const int32_t *ids, int64_t P, int32_t T,
                      uint32_t *lists)
{
    for (int64_t i = 0; i < m; i++)
        orc_sample_list(seed, ell, (uint32_t)ids[i], P, T, lists + i * T);
}

/* ------------------------------------------------------------------------ */
/* Conflict graph (Alg. 1 construct_conflict_graph; Sec. IV-A: an edge of the */
/* relation graph is conflicting when the two endpoints' lists intersect).    */
/* ------------------------------------------------------------------------ */

/* 1 if two sorted lists share a colour. */
static int lists_intersect(const uint32_t *a, const uint32_t *b, int T)
{
    int i = 0, j = 0;
    while (i < T && j < T) {
        if (a[i] == b[j]) return 1;
        if (a[i] < b[j]) i++;
        else j++;
    }
    return 0;
}

/* Smallest colour two sorted lists share, or UINT32_MAX if none. */
static uint32_t min_shared(const uint32_t *a, const uint32_t *b, int T)
{
    int i = 0, j = 0;
    while (i < T && j < T) {
        if (a[i] == b[j]) return a[i];
        if (a[i] < b[j]) i++;
        else j++;
    }
    return UINT32_MAX;
}

/* Growable edge array of (u, v) local-index pairs. */
typedef struct {
    int32_t *uv;
    int64_t count, cap;
} edge_buf;

static int edge_push(edge_buf *e, int32_t u, int32_t v)
{
    if (e->count == e->cap) {
        int64_t nc = e->cap ? e->cap * 2 : 1024;
        int32_t *p = (int32_t *)realloc(e->uv, (size_t)nc * 2 * sizeof(int32_t));
        if (!p) return -1;
        e->uv = p;
        e->cap = nc;
    }
    e->uv[2 * e->count] = u;
    e->uv[2 * e->count + 1] = v;
    e->count++;
    return 0;
}

static int cmp_edge(const void *pa, const void *pb)
{
    const int32_t *a = (const int32_t *)pa, *b = (const int32_t *)pb;
    if (a[0] != b[0]) return a[0] < b[0] ? -1 : 1;
    if (a[1] != b[1]) return a[1] < b[1] ? -1 : 1;
    return 0;
}

/* The definition written out: every pair a < b of the m vertices is an edge
 * iff the relation holds and their lists intersect.  `chars` holds the
 * decoded strings of ALL n vertices; ids maps local index -> original id.
 * Returns |E_c|; writes min(|E_c|, cap) pairs (a < b, lexicographic). */
int64_t orc_conflict_edges_allpairs(int32_t q, int64_t m, const int32_t *ids, const char *chars,
                                    const uint32_t *lists, int32_t T, int32_t rel, int32_t *out_uv,
                                    int64_t cap)
{
    int64_t count = 0;
    for (int64_t a = 0; a < m; a++)
        for (int64_t b = a + 1; b < m; b++) {
            if (!lists_intersect(lists + a * T, lists + b * T, T)) continue;
            if (!orc_relation_chars(q, chars + (int64_t)ids[a] * q, chars + (int64_t)ids[b] * q, rel))
                continue;
            if (count < cap) {
                out_uv[2 * count] = (int32_t)a;
                out_uv[2 * count + 1] = (int32_t)b;
            }
            count++;
        }
    return count;
}

/* The same edge set enumerated colour by colour: the vertices holding colour
 * c are the only candidates that conflict through c, and a pair sharing
 * several colours is recorded once, at the smallest shared colour.  Only
 * colours in [c_lo, c_hi) are visited (the whole palette by default), which
 * lets a caller time a bounded slice.  Edges are returned sorted; with
 * eb == NULL they are only counted.
 * *pair_tests receives sum over visited colours of C(|B_c|, 2). */
static int64_t conflict_edges_by_colour(int32_t q, int64_t m, const int32_t *ids, const char *chars,
                                        const uint32_t *lists, int32_t T, int64_t P, int32_t rel,
                                        int64_t c_lo, int64_t c_hi, edge_buf *eb, int64_t *pair_tests)
{
    int64_t *start = (int64_t *)calloc((size_t)P + 1, sizeof(int64_t));
    int32_t *members = (int32_t *)malloc((size_t)(m * T > 0 ? m * T : 1) * sizeof(int32_t));
    int64_t *fill = (int64_t *)calloc((size_t)P, sizeof(int64_t));
    if (!start || !members || !fill) {
        free(start); free(members); free(fill);
        return -1;
    }
    for (int64_t a = 0; a < m; a++)
        for (int k = 0; k < T; k++) start[lists[a * T + k] + 1]++;
    for (int64_t c = 0; c < P; c++) start[c + 1] += start[c];
    for (int64_t a = 0; a < m; a++) /* ascending a: each bucket is sorted */
        for (int k = 0; k < T; k++) {
            uint32_t c = lists[a * T + k];
            members[start[c] + fill[c]++] = (int32_t)a;
        }
    free(fill);
    int64_t tests = 0, counted = 0;
    if (c_lo < 0) c_lo = 0;
    if (c_hi > P) c_hi = P;
    for (int64_t c = c_lo; c < c_hi; c++) {
        int64_t s = start[c], e = start[c + 1];
        tests += (e - s) * (e - s - 1) / 2;
        for (int64_t i = s; i < e; i++)
            for (int64_t j = i + 1; j < e; j++) {
                int32_t a = members[i], b = members[j];
                if (!orc_relation_chars(q, chars + (int64_t)ids[a] * q, chars + (int64_t)ids[b] * q, rel))
                    continue;
                if (min_shared(lists + (int64_t)a * T, lists + (int64_t)b * T, T) != (uint32_t)c) continue;
                if (!eb) {
                    counted++;
                    continue;
                }
                if (edge_push(eb, a, b)) {
                    free(start); free(members);
                    return -1;
                }
            }
    }
    free(start);
    free(members);
    if (pair_tests) *pair_tests = tests;
    if (!eb) return counted;
    qsort(eb->uv, (size_t)eb->count, 2 * sizeof(int32_t), cmp_edge);
    return eb->count;
}

/* Exported wrapper: returns |E_c| over the colour slice, copies up to cap
 * sorted pairs.  Returns -1 on allocation failure. */
int64_t orc_conflict_edges_bucketed(int32_t q, int64_t m, const int32_t *ids, const char *chars,
                                    const uint32_t *lists, int32_t T, int64_t P, int32_t rel,
                                    int64_t c_lo, int64_t c_hi, int32_t *out_uv, int64_t cap,
                                    int64_t *pair_tests)
{
    edge_buf eb = {0, 0, 0};
    int64_t cnt = conflict_edges_by_colour(q, m, ids, chars, lists, T, P, rel, c_lo, c_hi, &eb, pair_tests);
    if (cnt >= 0 && out_uv) {
        int64_t k = cnt < cap ? cnt : cap;
        memcpy(out_uv, eb.uv, (size_t)k * 2 * sizeof(int32_t));
    }
    free(eb.uv);
    return cnt;
}

/* Exported: |E_c| over the colour slice [c_lo, c_hi) without storing any
 * edge (the same enumeration, counting only). */
int64_t orc_count_conflict_edges(int32_t q, int64_t m, const int32_t *ids, const char *chars,
                                 const uint32_t *lists, int32_t T, int64_t P, int32_t rel, int64_t c_lo,
                                 int64_t c_hi, int64_t *pair_tests)
{
    return conflict_edges_by_colour(q, m, ids, chars, lists, T, P, rel, c_lo, c_hi, NULL, pair_tests);
}

/* ------------------------------------------------------------------------ */
/* List colouring of the conflict graph in a static random order (Sec. IV-B, */
/* static order schemes: each vertex in turn takes the first colour of its    */
/* list not already held by a neighbour; Alg. 1 also gives unconflicted       */
/* vertices a colour of their list -- here the first one).                   */
/* Vertices whose list is exhausted stay uncoloured (-1).                     */
/* ------------------------------------------------------------------------ */
static const uint64_t *g_sort_prio; /* qsort context (single-threaded) */

static int cmp_order(const void *pa, const void *pb)
{
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    if (g_sort_prio[a] != g_sort_prio[b]) return g_sort_prio[a] < g_sort_prio[b] ? -1 : 1;
    return a < b ? -1 : (a > b ? 1 : 0);
}

/* prio[m]: priorities; local index order equals original-id order, so the
 * (prio, index) order is the (prio, id) order.  CSR (rowptr, adj) is the
 * symmetric conflict graph.  col[m] receives palette colours or -1. */
int32_t orc_greedy_list_color(int64_t m, const uint64_t *prio, const uint32_t *lists, int32_t T, int64_t P,
                              const int64_t *rowptr, const int32_t *adj, int32_t *col)
{
    int64_t *order = (int64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
    int64_t *rank = (int64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
    int64_t *mark = (int64_t *)malloc((size_t)P * sizeof(int64_t));
    if (!order || !rank || !mark) {
        free(order); free(rank); free(mark);
        return -1;
    }
    for (int64_t i = 0; i < m; i++) order[i] = i;
    g_sort_prio = prio;
    qsort(order, (size_t)m, sizeof(int64_t), cmp_order);
    for (int64_t r = 0; r < m; r++) rank[order[r]] = r;
    for (int64_t c = 0; c < P; c++) mark[c] = -1;
    for (int64_t i = 0; i < m; i++) col[i] = -1;
    for (int64_t r = 0; r < m; r++) {
        int64_t v = order[r];
        for (int64_t e = rowptr[v]; e < rowptr[v + 1]; e++) {
            int64_t u = adj[e];
            if (rank[u] < rank[v] && col[u] >= 0) mark[col[u]] = v; /* forbidden for v */
        }
        for (int k = 0; k < T; k++) {
            uint32_t c = lists[v * T + k];
            if (mark[c] != v) {
                col[v] = (int32_t)c;
                break;
            }
        }
    }
    free(order);
    free(rank);
    free(mark);
    return 0;
}

/* Symmetric CSR from a sorted (a < b) edge list. */
static int build_csr(int64_t m, const int32_t *uv, int64_t ne, int64_t **rowptr_out, int32_t **adj_out)
{
    int64_t *rowptr = (int64_t *)calloc((size_t)m + 1, sizeof(int64_t));
    int32_t *adj = (int32_t *)malloc((size_t)(2 * ne > 0 ? 2 * ne : 1) * sizeof(int32_t));
    int64_t *pos = (int64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
    if (!rowptr || !adj || !pos) {
        free(rowptr); free(adj); free(pos);
        return -1;
    }
    for (int64_t e = 0; e < ne; e++) {
        rowptr[uv[2 * e] + 1]++;
        rowptr[uv[2 * e + 1] + 1]++;
    }
    for (int64_t i = 0; i < m; i++) rowptr[i + 1] += rowptr[i];
    for (int64_t i = 0; i < m; i++) pos[i] = rowptr[i];
    for (int64_t e = 0; e < ne; e++) {
        int32_t a = uv[2 * e], b = uv[2 * e + 1];
        adj[pos[a]++] = b;
        adj[pos[b]++] = a;
    }
    free(pos);
    *rowptr_out = rowptr;
    *adj_out = adj;
    return 0;
}

/* Exported: greedy on an edge list (for tests that supply their own graph). */
int32_t orc_greedy_from_edges(int64_t m, const uint64_t *prio, const uint32_t *lists, int32_t T, int64_t P,
                              const int32_t *uv, int64_t ne, int32_t *col)
{
    int64_t *rowptr;
    int32_t *adj;
    if (build_csr(m, uv, ne, &rowptr, &adj)) return -1;
    int32_t rc = orc_greedy_list_color(m, prio, lists, T, P, rowptr, adj, col);
    free(rowptr);
    free(adj);
    return rc;
}

/* The same static-order greedy without the conflict graph.  When v's turn
 * comes, colour c of its list is forbidden exactly when an earlier vertex u
 * with {u, v} in E_c already holds c.  Such a u took c from its own list, so
 * c lies in both lists and the pair is in E_c iff the relation holds.  Hence
 * c is forbidden iff some vertex already coloured c (all of them come
 * earlier) is related to v: the test needs the colour classes built so far
 * and the relation, nothing else.  chars holds the decoded strings of all
 * vertices, ids maps local index -> original id, prio[m] the priorities.
 * col[m] receives palette colours or -1.  Returns 0, or -1 on allocation
 * failure. */
int32_t orc_greedy_by_classes(int32_t q, int64_t m, const int32_t *ids, const char *chars, const uint32_t *lists,
                              int32_t T, int64_t P, const uint64_t *prio, int32_t rel, int32_t *col)
{
    int64_t *order = (int64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
    int64_t *head = (int64_t *)malloc((size_t)(P > 0 ? P : 1) * sizeof(int64_t));
    int64_t *next = (int64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
    if (!order || !head || !next) {
        free(order); free(head); free(next);
        return -1;
    }
    for (int64_t i = 0; i < m; i++) order[i] = i;
    g_sort_prio = prio;
    qsort(order, (size_t)m, sizeof(int64_t), cmp_order);
    for (int64_t c = 0; c < P; c++) head[c] = -1; /* class of c: a linked list of its vertices */
    for (int64_t i = 0; i < m; i++) col[i] = -1;
    for (int64_t r = 0; r < m; r++) {
        int64_t v = order[r];
        const char *sv = chars + (int64_t)ids[v] * q;
        for (int k = 0; k < T; k++) {
            uint32_t c = lists[v * T + k];
            int forbidden = 0;
            for (int64_t u = head[c]; u >= 0 && !forbidden; u = next[u])
                forbidden = orc_relation_chars(q, chars + (int64_t)ids[u] * q, sv, rel);
            if (!forbidden) {
                col[v] = (int32_t)c;
                next[v] = head[c];
                head[c] = v;
                break;
            }
        }
    }
    free(order);
    free(head);
    free(next);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Dynamic-order list colouring (Alg. 2, Sec. IV-B): the vertex with the     */
/* shortest remaining list goes next, and the colour it takes is removed     */
/* from its uncoloured neighbours' lists.  A vertex whose list empties stays  */
/* uncoloured for the next iteration.                                        */
/* Readings where the algorithm leaves a choice open:                        */
/*  - vertices sit in one array per remaining list size; the arrays start in */
/*    ascending vertex order, a removal moves the array's last vertex into   */
/*    the hole, and a vertex whose list shrinks is appended to its new array;*/
/*  - step k (k = 0, 1, ...) draws r0 = H(seed; k, 0, ell, "DYNV") and picks  */
/*    entry floor(r0 * count / 2^64) of the lowest non-empty array, then     */
/*    r1 = H(seed; k, 1, ell, "DYNV") picks entry floor(r1 * size / 2^64) of */
/*    that vertex's remaining list, kept in ascending colour order.          */
/* ------------------------------------------------------------------------ */
#define ORC_TAG_DYNV 0x44594E56u

/* col[m] receives list colours or -1; order[m] (may be NULL) the vertices in
 * the order they were taken (coloured or emptied), -1-terminated if fewer.
 * Returns the number of coloured vertices, or -1 on allocation failure. */
static int64_t greedy_dynamic_csr(int64_t m, const uint32_t *lists, int32_t T, const int64_t *rowptr,
                                  const int32_t *adj, uint64_t seed, uint32_t ell, int32_t *col, int32_t *order)
{
    uint32_t *cl = (uint32_t *)malloc((size_t)(m * T > 0 ? m * T : 1) * sizeof(uint32_t));
    int32_t *sz = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    int64_t *where = (int64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
    int32_t *arr = (int32_t *)malloc((size_t)((T + 1) * (m > 0 ? m : 1)) * sizeof(int32_t));
    int64_t *cnt = (int64_t *)calloc((size_t)(T + 1), sizeof(int64_t));
    char *done = (char *)calloc((size_t)(m > 0 ? m : 1), 1);
    if (!cl || !sz || !where || !arr || !cnt || !done) {
        free(cl); free(sz); free(where); free(arr); free(cnt); free(done);
        return -1;
    }
    memcpy(cl, lists, (size_t)(m * T) * sizeof(uint32_t));
    for (int64_t v = 0; v < m; v++) {
        col[v] = -1;
        if (order) order[v] = -1;
        sz[v] = T;
        where[v] = cnt[T];
        arr[(int64_t)T * m + cnt[T]++] = (int32_t)v;
    }
    int64_t taken = 0, colored = 0;
    for (uint32_t step = 0; taken < m; step++) {
        int32_t s = 1;
        while (s <= T && cnt[s] == 0) s++;
        if (s > T) break; /* every vertex is taken */
        uint64_t r0 = orc_hash64(seed, step, 0, ell, ORC_TAG_DYNV);
        int64_t at = (int64_t)mul_high64(r0, (uint64_t)cnt[s]);
        int32_t v = arr[(int64_t)s * m + at];
        /* remove v from its array */
        int32_t last = arr[(int64_t)s * m + cnt[s] - 1];
        arr[(int64_t)s * m + at] = last;
        where[last] = at;
        cnt[s]--;
        done[v] = 1;
        if (order) order[taken] = v;
        taken++;
        uint64_t r1 = orc_hash64(seed, step, 1, ell, ORC_TAG_DYNV);
        uint32_t c = cl[v * T + (int64_t)mul_high64(r1, (uint64_t)sz[v])];
        col[v] = (int32_t)c;
        colored++;
        for (int64_t e = rowptr[v]; e < rowptr[v + 1]; e++) {
            int32_t u = adj[e];
            if (done[u]) continue;
            uint32_t *lu = cl + (int64_t)u * T;
            int32_t k = 0;
            while (k < sz[u] && lu[k] != c) k++;
            if (k == sz[u]) continue; /* c is not (or no longer) in u's list */
            for (int32_t j = k; j + 1 < sz[u]; j++) lu[j] = lu[j + 1];
            /* move u from array sz[u] to array sz[u] - 1 (or take it out) */
            int32_t su = sz[u];
            int32_t lastu = arr[(int64_t)su * m + cnt[su] - 1];
            arr[(int64_t)su * m + where[u]] = lastu;
            where[lastu] = where[u];
            cnt[su]--;
            sz[u] = su - 1;
            if (sz[u] == 0) {
                done[u] = 1;
                if (order) order[taken] = u;
                taken++;
            } else {
                where[u] = cnt[sz[u]];
                arr[(int64_t)sz[u] * m + cnt[sz[u]]++] = u;
            }
        }
    }
    free(cl); free(sz); free(where); free(arr); free(cnt); free(done);
    return colored;
}

/* Exported: Alg. 2 on an edge list (for tests that supply their own graph). */
int64_t orc_greedy_dynamic(int64_t m, const uint32_t *lists, int32_t T, const int32_t *uv, int64_t ne,
                           uint64_t seed, uint32_t ell, int32_t *col, int32_t *order)
{
    int64_t *rowptr;
    int32_t *adj;
    if (build_csr(m, uv, ne, &rowptr, &adj)) return -1;
    int64_t rc = greedy_dynamic_csr(m, lists, T, rowptr, adj, seed, ell, col, order);
    free(rowptr);
    free(adj);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* A round form of Alg. 2 for parallel execution.  Alg. 2 takes one vertex   */
/* at a time, the one with the shortest remaining list, gives it a random    */
/* colour of its list and removes that colour from its neighbours' lists.   */
/* Here many vertices move per round (a reading for parallel hardware; the  */
/* result differs from the sequential order, so it has its own oracle):     */
/*  1. active vertices: uncoloured and not failed; one whose list is empty   */
/*     fails (stays uncoloured for the next iteration of Alg. 1);           */
/*  2. R = max(ceil(A / divisor), min(A, 64)) of the A active vertices      */
/*     request a colour: those with the shortest lists, by the smallest     */
/*     size s* whose cumulative count reaches R; of the vertices with       */
/*     exactly s* colours left, those whose key h = high 32 bits of         */
/*     H(seed; id, round, ell, "DYNK") is below cut = floor(need 2^32 / eq) */
/*     (need = R minus the vertices with fewer colours, eq = the vertices   */
/*     with exactly s*; need = eq takes all of them);                       */
/*  3. a requester asks for entry floor(r size / 2^64) of its remaining     */
/*     list in ascending colour order, r = H(seed; id, round, ell, "DYNC");  */
/*  4. each colour's requesters, in ascending (size, h, vertex) order, take */
/*     the colour unless a conflict neighbour took it earlier in this       */
/*     order (requesters of one colour share it, so conflict = relation);  */
/*  5. every conflict neighbour of a vertex that took colour c loses c from */
/*     its list.                                                            */
/* id is the vertex's original id, so the result does not depend on where  */
/* the vertex sits in the iteration's vertex set.                          */
/* ------------------------------------------------------------------------ */
#define ORC_TAG_DYNK 0x44594E4Bu
#define ORC_TAG_DYNC 0x44594E43u

typedef struct {
    uint32_t colour;
    uint64_t key;
    int32_t v;
} orc_request;

static int cmp_request(const void *a, const void *b)
{
    const orc_request *x = (const orc_request *)a, *y = (const orc_request *)b;
    if (x->colour != y->colour) return x->colour < y->colour ? -1 : 1;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return (x->v > y->v) - (x->v < y->v);
}

static int64_t greedy_rounds_csr(int64_t m, const int32_t *ids, const uint32_t *lists, int32_t T,
                                 const int64_t *rowptr, const int32_t *adj, uint64_t seed, uint32_t ell,
                                 int32_t divisor, int32_t *col, int32_t *n_rounds)
{
    char *alive = (char *)malloc((size_t)(m * T > 0 ? m * T : 1));
    int32_t *size = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    char *failed = (char *)calloc((size_t)(m > 0 ? m : 1), 1);
    int32_t *took = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t)); /* round it took its colour */
    int64_t *hist = (int64_t *)malloc((size_t)(T + 1) * sizeof(int64_t));
    orc_request *req = (orc_request *)malloc((size_t)(m > 0 ? m : 1) * sizeof(orc_request));
    if (!alive || !size || !failed || !took || !hist || !req) {
        free(alive); free(size); free(failed); free(took); free(hist); free(req);
        return -1;
    }
    for (int64_t i = 0; i < m * T; i++) alive[i] = 1;
    for (int64_t v = 0; v < m; v++) {
        size[v] = T;
        col[v] = -1;
        took[v] = -1;
    }
    int64_t colored = 0;
    int32_t round = 0;
    for (;; round++) {
        int64_t A = 0;
        for (int32_t s = 0; s <= T; s++) hist[s] = 0;
        for (int64_t v = 0; v < m; v++) {
            if (col[v] >= 0 || failed[v]) continue;
            if (size[v] == 0) {
                failed[v] = 1;
                continue;
            }
            hist[size[v]]++;
            A++;
        }
        if (A == 0) break;
        int64_t R = (A + divisor - 1) / divisor;
        const int64_t floor_r = A < 64 ? A : 64;
        if (R < floor_r) R = floor_r;
        int64_t below = 0, eq = 0;
        int32_t sstar = T;
        for (int32_t s = 1; s <= T; s++) {
            if (below + hist[s] >= R) {
                sstar = s;
                eq = hist[s];
                break;
            }
            below += hist[s];
        }
        const int64_t need = R - below;
        const uint64_t cut = need >= eq ? ((uint64_t)1 << 32) : ((uint64_t)need << 32) / (uint64_t)eq;
        int64_t nreq = 0;
        for (int64_t v = 0; v < m; v++) {
            if (col[v] >= 0 || failed[v]) continue;
            const uint64_t h = orc_hash64(seed, (uint32_t)ids[v], (uint32_t)round, ell, ORC_TAG_DYNK) >> 32;
            if (!(size[v] < sstar || (size[v] == sstar && h < cut))) continue;
            const uint64_t r = orc_hash64(seed, (uint32_t)ids[v], (uint32_t)round, ell, ORC_TAG_DYNC);
            int64_t j = (int64_t)mul_high64(r, (uint64_t)size[v]);
            int32_t k = 0;
            for (; k < T; k++)
                if (alive[v * T + k] && j-- == 0) break;
            req[nreq].colour = lists[v * T + k];
            req[nreq].key = ((uint64_t)size[v] << 32) | h;
            req[nreq].v = (int32_t)v;
            nreq++;
        }
        qsort(req, (size_t)nreq, sizeof(orc_request), cmp_request);
        for (int64_t i = 0; i < nreq; i++) {
            const int32_t u = req[i].v;
            const uint32_t c = req[i].colour;
            int ok = 1;
            for (int64_t e = rowptr[u]; e < rowptr[u + 1] && ok; e++) {
                const int32_t w = adj[e];
                if (took[w] == round && col[w] == (int32_t)c) ok = 0;
            }
            if (ok) {
                col[u] = (int32_t)c;
                took[u] = round;
                colored++;
            }
        }
        for (int64_t i = 0; i < nreq; i++) {
            const int32_t u = req[i].v;
            if (took[u] != round) continue;
            const uint32_t c = (uint32_t)col[u];
            for (int64_t e = rowptr[u]; e < rowptr[u + 1]; e++) {
                const int32_t w = adj[e];
                for (int32_t k = 0; k < T; k++)
                    if (lists[(int64_t)w * T + k] == c) {
                        if (alive[(int64_t)w * T + k]) {
                            alive[(int64_t)w * T + k] = 0;
                            size[w]--;
                        }
                        break;
                    }
            }
        }
    }
    if (n_rounds) *n_rounds = round;
    free(alive); free(size); free(failed); free(took); free(hist); free(req);
    return colored;
}

/* Exported: the round form on an edge list (for tests that supply their own
 * graph).  ids[m]: the vertices' original ids (they key the draws). */
int64_t orc_greedy_dynamic_rounds(int64_t m, const int32_t *ids, const uint32_t *lists, int32_t T, const int32_t *uv,
                                  int64_t ne, uint64_t seed, uint32_t ell, int32_t divisor, int32_t *col,
                                  int32_t *n_rounds)
{
    int64_t *rowptr;
    int32_t *adj;
    if (divisor < 1 || build_csr(m, uv, ne, &rowptr, &adj)) return -1;
    int64_t rc = greedy_rounds_csr(m, ids, lists, T, rowptr, adj, seed, ell, divisor, col, n_rounds);
    free(rowptr);
    free(adj);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* The iteration (Alg. 1): estimate (P, T), draw lists, build the conflict    */
/* graph, colour it, and recurse on the uncoloured vertices with a fresh      */
/* palette.  Reading of the garbled palette indices: iteration ell uses the  */
/* half-open range [offset, offset + P_ell), offset = sum of earlier P.       */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t m, P, T, pair_tests, edges, colored, offset;
} orc_iter_stat;

/* Returns the number of distinct colours, or -1 on allocation failure.
 * out_colors[n] receives global colour ids.  stats (may be NULL) receives
 * up to max_stats per-iteration records; *n_iters the iteration count. */
static int64_t color_driver(int64_t n, int32_t q, const uint64_t *x, const uint64_t *z, uint64_t seed,
                            double frac, double alpha, int32_t rel, int32_t fixed_T, int32_t dynamic,
                            int32_t divisor, int32_t *out_colors, orc_iter_stat *stats, int32_t max_stats,
                            int32_t *n_iters);

int64_t orc_color(int64_t n, int32_t q, const uint64_t *x, const uint64_t *z, uint64_t seed, double frac,
                  double alpha, int32_t rel, int32_t fixed_T, int32_t *out_colors, orc_iter_stat *stats,
                  int32_t max_stats, int32_t *n_iters)
{
    return color_driver(n, q, x, z, seed, frac, alpha, rel, fixed_T, 0, 0, out_colors, stats, max_stats, n_iters);
}

/* Alg. 1 with the dynamic-order colourer of Alg. 2 in place of the static
 * random order. */
int64_t orc_color_dynamic(int64_t n, int32_t q, const uint64_t *x, const uint64_t *z, uint64_t seed, double frac,
                          double alpha, int32_t rel, int32_t fixed_T, int32_t *out_colors, orc_iter_stat *stats,
                          int32_t max_stats, int32_t *n_iters)
{
    return color_driver(n, q, x, z, seed, frac, alpha, rel, fixed_T, 1, 0, out_colors, stats, max_stats, n_iters);
}

/* Alg. 1 with the round form of Alg. 2 (divisor >= 1: about one active
 * vertex in `divisor` requests a colour per round). */
int64_t orc_color_dynamic_rounds(int64_t n, int32_t q, const uint64_t *x, const uint64_t *z, uint64_t seed,
                                 double frac, double alpha, int32_t rel, int32_t fixed_T, int32_t divisor,
                                 int32_t *out_colors, orc_iter_stat *stats, int32_t max_stats, int32_t *n_iters)
{
    if (divisor < 1) return -1;
    return color_driver(n, q, x, z, seed, frac, alpha, rel, fixed_T, 2, divisor, out_colors, stats, max_stats,
                        n_iters);
}

static int64_t color_driver(int64_t n, int32_t q, const uint64_t *x, const uint64_t *z, uint64_t seed,
                            double frac, double alpha, int32_t rel, int32_t fixed_T, int32_t dynamic,
                            int32_t divisor, int32_t *out_colors, orc_iter_stat *stats, int32_t max_stats,
                            int32_t *n_iters)
{
    char *chars = (char *)malloc((size_t)(n * q > 0 ? n * q : 1));
    int32_t *ids = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!chars || !ids) {
        free(chars); free(ids);
        return -1;
    }
    orc_decode(n, q, x, z, chars);
    for (int64_t i = 0; i < n; i++) {
        ids[i] = (int32_t)i;
        out_colors[i] = -1;
    }
    int64_t m = n, offset = 0, distinct = 0;
    uint32_t ell = 1;
    int32_t it = 0;
    while (m > 0) {
        int64_t P;
        int32_t T;
        orc_params(m, frac, alpha, fixed_T, &P, &T);
        uint32_t *lists = (uint32_t *)malloc((size_t)(m * T) * sizeof(uint32_t));
        uint64_t *prio = (uint64_t *)malloc((size_t)m * sizeof(uint64_t));
        int32_t *col = (int32_t *)malloc((size_t)m * sizeof(int32_t));
        char *used = (char *)calloc((size_t)P, 1);
        if (!lists || !prio || !col || !used) {
            free(lists); free(prio); free(col); free(used); free(chars); free(ids);
            return -1;
        }
        orc_sample_lists(seed, ell, m, ids, P, T, lists);
        for (int64_t i = 0; i < m; i++) prio[i] = orc_priority(seed, ell, (uint32_t)ids[i]);
        edge_buf eb = {0, 0, 0};
        int64_t tests = 0;
        int64_t ne = conflict_edges_by_colour(q, m, ids, chars, lists, T, P, rel, 0, P, &eb, &tests);
        int failed = ne < 0;
        if (!failed && dynamic == 2)
            failed = orc_greedy_dynamic_rounds(m, ids, lists, T, eb.uv, ne, seed, ell, divisor, col, NULL) < 0;
        else if (!failed && dynamic) failed = orc_greedy_dynamic(m, lists, T, eb.uv, ne, seed, ell, col, NULL) < 0;
        else if (!failed) failed = orc_greedy_from_edges(m, prio, lists, T, P, eb.uv, ne, col) != 0;
        if (failed) {
            free(eb.uv); free(lists); free(prio); free(col); free(used); free(chars); free(ids);
            return -1;
        }
        free(eb.uv);
        int64_t next = 0, colored = 0;
        for (int64_t i = 0; i < m; i++) {
            if (col[i] >= 0) {
                out_colors[ids[i]] = (int32_t)(offset + col[i]);
                if (!used[col[i]]) {
                    used[col[i]] = 1;
                    distinct++;
                }
                colored++;
            } else {
                ids[next++] = ids[i]; /* ascending order is kept */
            }
        }
        if (stats && it < max_stats) {
            orc_iter_stat s = {m, P, T, tests, ne, colored, offset};
            stats[it] = s;
        }
        it++;
        free(lists);
        free(prio);
        free(col);
        free(used);
        offset += P;
        m = next;
        ell++;
    }
    if (n_iters) *n_iters = it;
    free(chars);
    free(ids);
    return distinct;
}

/* ------------------------------------------------------------------------ */
/* Iterations with a parameter schedule: iteration ell uses (fracs[ell-1],   */
/* alphas[ell-1]) (the last entry once the schedule is exhausted).  This is */
/* how a learned predictor's per-iteration outputs are replayed.            */
/* ------------------------------------------------------------------------ */
int64_t orc_color_schedule(int64_t n, int32_t q, const uint64_t *x, const uint64_t *z, uint64_t seed,
                           const double *fracs, const double *alphas, int32_t n_sched, int32_t rel,
                           int32_t *out_colors, orc_iter_stat *stats, int32_t max_stats, int32_t *n_iters)
{
    char *chars = (char *)malloc((size_t)(n * q > 0 ? n * q : 1));
    int32_t *ids = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!chars || !ids || n_sched < 1) {
        free(chars); free(ids);
        return -1;
    }
    orc_decode(n, q, x, z, chars);
    for (int64_t i = 0; i < n; i++) {
        ids[i] = (int32_t)i;
        out_colors[i] = -1;
    }
    int64_t m = n, offset = 0, distinct = 0;
    uint32_t ell = 1;
    int32_t it = 0;
    while (m > 0) {
        const int32_t si = (int32_t)ell - 1 < n_sched ? (int32_t)ell - 1 : n_sched - 1;
        int64_t P;
        int32_t T;
        orc_params(m, fracs[si], alphas[si], 0, &P, &T);
        uint32_t *lists = (uint32_t *)malloc((size_t)(m * T) * sizeof(uint32_t));
        uint64_t *prio = (uint64_t *)malloc((size_t)m * sizeof(uint64_t));
        int32_t *col = (int32_t *)malloc((size_t)m * sizeof(int32_t));
        char *used = (char *)calloc((size_t)P, 1);
        if (!lists || !prio || !col || !used) {
            free(lists); free(prio); free(col); free(used); free(chars); free(ids);
            return -1;
        }
        orc_sample_lists(seed, ell, m, ids, P, T, lists);
        for (int64_t i = 0; i < m; i++) prio[i] = orc_priority(seed, ell, (uint32_t)ids[i]);
        edge_buf eb = {0, 0, 0};
        int64_t tests = 0;
        int64_t ne = conflict_edges_by_colour(q, m, ids, chars, lists, T, P, rel, 0, P, &eb, &tests);
        if (ne < 0 || orc_greedy_from_edges(m, prio, lists, T, P, eb.uv, ne, col)) {
            free(eb.uv); free(lists); free(prio); free(col); free(used); free(chars); free(ids);
            return -1;
        }
        free(eb.uv);
        int64_t next = 0, colored = 0;
        for (int64_t i = 0; i < m; i++) {
            if (col[i] >= 0) {
                out_colors[ids[i]] = (int32_t)(offset + col[i]);
                if (!used[col[i]]) {
                    used[col[i]] = 1;
                    distinct++;
                }
                colored++;
            } else {
                ids[next++] = ids[i];
            }
        }
        if (stats && it < max_stats) {
            orc_iter_stat s = {m, P, T, tests, ne, colored, offset};
            stats[it] = s;
        }
        it++;
        free(lists); free(prio); free(col); free(used);
        offset += P;
        m = next;
        ell++;
    }
    if (n_iters) *n_iters = it;
    free(chars);
    free(ids);
    return distinct;
}

/* ------------------------------------------------------------------------ */
/* Alg. 1 without storing any conflict graph: each iteration colours by the  */
/* colour classes (orc_greedy_by_classes), so memory stays O(n q + m T) and  */
/* the largest workloads fit a host.  Iteration ell uses (fracs[ell-1],      */
/* alphas[ell-1]), the last entry after the end (n_sched = 1: fixed          */
/* parameters).  With count_edges = 0 the per-iteration |E_c| is not counted */
/* (stats carry -1); otherwise it is counted colour by colour, as above.    */
/* ------------------------------------------------------------------------ */
static int32_t learned_params(const double *mlp, double beta, const char *chars, int32_t q, int64_t m,
                              const int32_t *ids, uint64_t seed, uint32_t ell, int32_t rel, double *frac,
                              double *alpha);

static int64_t classes_driver(int64_t n, int32_t q, const uint64_t *x, const uint64_t *z, uint64_t seed,
                              const double *fracs, const double *alphas, int32_t n_sched, const double *mlp,
                              double beta, int32_t rel, int32_t fixed_T, int32_t count_edges, int32_t *out_colors,
                              orc_iter_stat *stats, int32_t max_stats, int32_t *n_iters, double *sched,
                              int32_t max_sched)
{
    char *chars = (char *)malloc((size_t)(n * q > 0 ? n * q : 1));
    int32_t *ids = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!chars || !ids) {
        free(chars); free(ids);
        return -1;
    }
    orc_decode(n, q, x, z, chars);
    for (int64_t i = 0; i < n; i++) {
        ids[i] = (int32_t)i;
        out_colors[i] = -1;
    }
    int64_t m = n, offset = 0, distinct = 0;
    uint32_t ell = 1;
    int32_t it = 0;
    while (m > 0) {
        double frac, alpha;
        if (mlp) {
            learned_params(mlp, beta, chars, q, m, ids, seed, ell, rel, &frac, &alpha);
        } else {
            const int32_t si = (int32_t)ell - 1 < n_sched ? (int32_t)ell - 1 : n_sched - 1;
            frac = fracs[si];
            alpha = alphas[si];
        }
        if (sched && it < max_sched) {
            sched[2 * it] = frac;
            sched[2 * it + 1] = alpha;
        }
        int64_t P;
        int32_t T;
        orc_params(m, frac, alpha, fixed_T, &P, &T);
        uint32_t *lists = (uint32_t *)malloc((size_t)(m * T) * sizeof(uint32_t));
        uint64_t *prio = (uint64_t *)malloc((size_t)m * sizeof(uint64_t));
        int32_t *col = (int32_t *)malloc((size_t)m * sizeof(int32_t));
        char *used = (char *)calloc((size_t)P, 1);
        if (!lists || !prio || !col || !used) {
            free(lists); free(prio); free(col); free(used); free(chars); free(ids);
            return -1;
        }
        orc_sample_lists(seed, ell, m, ids, P, T, lists);
        for (int64_t i = 0; i < m; i++) prio[i] = orc_priority(seed, ell, (uint32_t)ids[i]);
        int64_t ne = -1, tests = 0;
        if (count_edges) {
            ne = conflict_edges_by_colour(q, m, ids, chars, lists, T, P, rel, 0, P, NULL, &tests);
        } else {
            /* pair tests from the bucket sizes alone */
            int64_t *cnt = (int64_t *)calloc((size_t)P, sizeof(int64_t));
            if (cnt) {
                for (int64_t e = 0; e < m * T; e++) cnt[lists[e]]++;
                for (int64_t c = 0; c < P; c++) tests += cnt[c] * (cnt[c] - 1) / 2;
            }
            free(cnt);
            if (!cnt) ne = -2;
        }
        if (ne == -2 || (count_edges && ne < 0) ||
            orc_greedy_by_classes(q, m, ids, chars, lists, T, P, prio, rel, col)) {
            free(lists); free(prio); free(col); free(used); free(chars); free(ids);
            return -1;
        }
        int64_t next = 0, colored = 0;
        for (int64_t i = 0; i < m; i++) {
            if (col[i] >= 0) {
                out_colors[ids[i]] = (int32_t)(offset + col[i]);
                if (!used[col[i]]) {
                    used[col[i]] = 1;
                    distinct++;
                }
                colored++;
            } else {
                ids[next++] = ids[i];
            }
        }
        if (stats && it < max_stats) {
            orc_iter_stat s = {m, P, T, tests, ne, colored, offset};
            stats[it] = s;
        }
        it++;
        free(lists); free(prio); free(col); free(used);
        offset += P;
        m = next;
        ell++;
    }
    if (n_iters) *n_iters = it;
    free(chars);
    free(ids);
    return distinct;
}

int64_t orc_color_classes(int64_t n, int32_t q, const uint64_t *x, const uint64_t *z, uint64_t seed,
                          const double *fracs, const double *alphas, int32_t n_sched, int32_t rel, int32_t fixed_T,
                          int32_t count_edges, int32_t *out_colors, orc_iter_stat *stats, int32_t max_stats,
                          int32_t *n_iters)
{
    if (n_sched < 1) return -1;
    return classes_driver(n, q, x, z, seed, fracs, alphas, n_sched, NULL, 0.0, rel, fixed_T, count_edges, out_colors,
                          stats, max_stats, n_iters, NULL, 0);
}

/* ------------------------------------------------------------------------ */
/* Instance features for the parameter predictor (the paper's Sec. VI       */
/* predicts (P', alpha) from the graph; here from five numbers per          */
/* iteration):                                                              */
/*   f0 = ln m, f1 = q, f2 = mean Pauli weight (non-identity positions per  */
/*   string), f3 = fraction of K sampled vertex pairs joined by the         */
/*   relation, f4 = ell.                                                    */
/* Sampled pair k: a = floor(r1*m/2^64), b' = floor(r2*(m-1)/2^64),         */
/* b = b' + (b' >= a), with r1, r2 the keyed draws (seed; k, 0|1, ell,      */
/* tag "FEAT"): a uniform ordered pair of distinct vertices.                */
/* ------------------------------------------------------------------------ */
#define ORC_TAG_FEAT 0x46454154u

void orc_features(int32_t q, const char *chars, int64_t m, const int32_t *ids, uint64_t seed, uint32_t ell,
                  int32_t rel, int32_t K, double out[5])
{
    int64_t weight = 0;
    for (int64_t i = 0; i < m; i++)
        for (int k = 0; k < q; k++)
            if (chars[(int64_t)ids[i] * q + k] != 'I') weight++;
    int64_t hits = 0;
    if (m >= 2)
        for (int32_t k = 0; k < K; k++) {
            uint64_t r1 = orc_hash64(seed, (uint32_t)k, 0, ell, ORC_TAG_FEAT);
            uint64_t r2 = orc_hash64(seed, (uint32_t)k, 1, ell, ORC_TAG_FEAT);
            uint64_t a = mul_high64(r1, (uint64_t)m);
            uint64_t b = mul_high64(r2, (uint64_t)(m - 1));
            if (b >= a) b++;
            hits += orc_relation_chars(q, chars + (int64_t)ids[a] * q, chars + (int64_t)ids[b] * q, rel);
        }
    out[0] = m > 0 ? log((double)m) : 0.0;
    out[1] = (double)q;
    out[2] = m > 0 ? (double)weight / (double)m : 0.0;
    out[3] = (m >= 2 && K > 0) ? (double)hits / (double)K : 0.0;
    out[4] = (double)ell;
}

/* Exported wrapper on bit-plane input. */
void orc_features_bits(int64_t n, int32_t q, const uint64_t *x, const uint64_t *z, int64_t m, const int32_t *ids,
                       uint64_t seed, uint32_t ell, int32_t rel, int32_t K, double out[5])
{
    char *chars = (char *)malloc((size_t)(n * q > 0 ? n * q : 1));
    if (!chars) return;
    orc_decode(n, q, x, z, chars);
    orc_features(q, chars, m, ids, seed, ell, rel, K, out);
    free(chars);
}

/* ------------------------------------------------------------------------ */
/* The parameter predictor: a 3-layer perceptron 6 -> 64 -> 64 -> 2 with    */
/* ReLU hidden layers (FP64 twin of the GPU network).  Its inputs are the   */
/* five features of the iteration's vertex set and the trade-off weight     */
/* beta of the bi-objective (Sec. VI, Eq. 7: the regressor is given the     */
/* graph and beta and predicts (P', alpha)).                                */
/* Parameter vector layout (4738 values):                                   */
/*   W1[64][6], b1[64], W2[64][64], b2[64], W3[2][64], b3[2]                */
/* Inputs are scaled before the first layer:                                */
/*   (ln m / 16, q / 128, weight / 128, density, ell / 16, beta).           */
/* Outputs o (2 values) map to parameters by                                */
/*   f = 0.01 + 0.24 sigmoid(o0), alpha = 1 + 3 sigmoid(o1).                */
/* Training loss over a batch of B rows: (1/(2B)) sum (o - t)^2.            */
/* ------------------------------------------------------------------------ */
#define ORC_H 64
#define ORC_IN 6
#define ORC_OUT 2
#define ORC_NPARAM (ORC_H * ORC_IN + ORC_H + ORC_H * ORC_H + ORC_H + ORC_OUT * ORC_H + ORC_OUT)

int32_t orc_mlp_nparams(void) { return ORC_NPARAM; }

static void mlp_scale(const double *raw, double *xin)
{
    xin[0] = raw[0] / 16.0;
    xin[1] = raw[1] / 128.0;
    xin[2] = raw[2] / 128.0;
    xin[3] = raw[3];
    xin[4] = raw[4] / 16.0;
    xin[5] = raw[5];
}

/* Forward pass of one row; keeps the activations for the gradient. */
static void mlp_row(const double *p, const double *raw, double *xin, double *h1, double *h2, double *o)
{
    const double *W1 = p, *b1 = W1 + ORC_H * ORC_IN, *W2 = b1 + ORC_H, *b2 = W2 + ORC_H * ORC_H;
    const double *W3 = b2 + ORC_H, *b3 = W3 + ORC_OUT * ORC_H;
    mlp_scale(raw, xin);
    for (int j = 0; j < ORC_H; j++) {
        double s = b1[j];
        for (int i = 0; i < ORC_IN; i++) s += W1[j * ORC_IN + i] * xin[i];
        h1[j] = s > 0.0 ? s : 0.0;
    }
    for (int j = 0; j < ORC_H; j++) {
        double s = b2[j];
        for (int i = 0; i < ORC_H; i++) s += W2[j * ORC_H + i] * h1[i];
        h2[j] = s > 0.0 ? s : 0.0;
    }
    for (int k = 0; k < ORC_OUT; k++) {
        double s = b3[k];
        for (int i = 0; i < ORC_H; i++) s += W3[k * ORC_H + i] * h2[i];
        o[k] = s;
    }
}

void orc_mlp_forward(const double *p, const double *raw, int32_t B, double *out)
{
    double xin[ORC_IN], h1[ORC_H], h2[ORC_H];
    for (int b = 0; b < B; b++) mlp_row(p, raw + (int64_t)b * ORC_IN, xin, h1, h2, out + (int64_t)b * ORC_OUT);
}

void orc_mlp_squash(const double *o, double *frac, double *alpha)
{
    *frac = 0.01 + 0.24 / (1.0 + exp(-o[0]));
    *alpha = 1.0 + 3.0 / (1.0 + exp(-o[1]));
}

/* Loss and its gradient by the chain rule (backpropagation). */
double orc_mlp_loss_grad(const double *p, const double *raw, const double *t, int32_t B, double *grad)
{
    const double *W2 = p + ORC_H * ORC_IN + ORC_H, *W3 = W2 + ORC_H * ORC_H + ORC_H;
    double *gW1 = grad, *gb1 = gW1 + ORC_H * ORC_IN, *gW2 = gb1 + ORC_H, *gb2 = gW2 + ORC_H * ORC_H;
    double *gW3 = gb2 + ORC_H, *gb3 = gW3 + ORC_OUT * ORC_H;
    for (int i = 0; i < ORC_NPARAM; i++) grad[i] = 0.0;
    double loss = 0.0;
    double xin[ORC_IN], h1[ORC_H], h2[ORC_H], o[ORC_OUT], d3[ORC_OUT], d2[ORC_H], d1[ORC_H];
    for (int b = 0; b < B; b++) {
        mlp_row(p, raw + (int64_t)b * ORC_IN, xin, h1, h2, o);
        for (int k = 0; k < ORC_OUT; k++) {
            const double e = o[k] - t[(int64_t)b * ORC_OUT + k];
            loss += 0.5 * e * e / B;
            d3[k] = e / B;
        }
        for (int i = 0; i < ORC_H; i++) {
            double s = 0.0;
            for (int k = 0; k < ORC_OUT; k++) s += W3[k * ORC_H + i] * d3[k];
            d2[i] = h2[i] > 0.0 ? s : 0.0;
        }
        for (int i = 0; i < ORC_H; i++) {
            double s = 0.0;
            for (int j = 0; j < ORC_H; j++) s += W2[j * ORC_H + i] * d2[j];
            d1[i] = h1[i] > 0.0 ? s : 0.0;
        }
        for (int k = 0; k < ORC_OUT; k++) {
            for (int i = 0; i < ORC_H; i++) gW3[k * ORC_H + i] += d3[k] * h2[i];
            gb3[k] += d3[k];
        }
        for (int j = 0; j < ORC_H; j++) {
            for (int i = 0; i < ORC_H; i++) gW2[j * ORC_H + i] += d2[j] * h1[i];
            gb2[j] += d2[j];
        }
        for (int j = 0; j < ORC_H; j++) {
            for (int i = 0; i < ORC_IN; i++) gW1[j * ORC_IN + i] += d1[j] * xin[i];
            gb1[j] += d1[j];
        }
    }
    return loss;
}

/* Adam (Kingma & Ba, 2015): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps). */
void orc_adam_step(double *p, const double *g, double *m, double *v, int32_t step, double lr, double b1, double b2,
                   double eps, int32_t nparam)
{
    const double c1 = 1.0 - pow(b1, (double)step), c2 = 1.0 - pow(b2, (double)step);
    for (int i = 0; i < nparam; i++) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        p[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
}

/* ------------------------------------------------------------------------ */
/* Alg. 1 with per-iteration parameters from the predictor (the FP64 twin): */
/* each iteration computes the features of its vertex set, runs the network */
/* and squashes its outputs to (f, alpha) in double, then proceeds as the   */
/* fixed-parameter run does (Sec. VI uses a predictor's (P', alpha) the     */
/* same way).  sched (may be NULL) receives the (f, alpha) of the first     */
/* max_sched iterations.                                                    */
/* ------------------------------------------------------------------------ */
static int32_t learned_params(const double *mlp, double beta, const char *chars, int32_t q, int64_t m,
                              const int32_t *ids, uint64_t seed, uint32_t ell, int32_t rel, double *frac,
                              double *alpha)
{
    double feat[ORC_IN], xin[ORC_IN], h1[ORC_H], h2[ORC_H], o[ORC_OUT];
    orc_features(q, chars, m, ids, seed, ell, rel, 4096, feat);
    feat[5] = beta;
    mlp_row(mlp, feat, xin, h1, h2, o);
    orc_mlp_squash(o, frac, alpha);
    return 0;
}

int64_t orc_color_learned(int64_t n, int32_t q, const uint64_t *x, const uint64_t *z, uint64_t seed,
                          const double *mlp, double beta, int32_t rel, int32_t count_edges, int32_t *out_colors,
                          orc_iter_stat *stats, int32_t max_stats, int32_t *n_iters, double *sched, int32_t max_sched)
{
    if (!mlp) return -1;
    return classes_driver(n, q, x, z, seed, NULL, NULL, 0, mlp, beta, rel, 0, count_edges, out_colors, stats, max_stats,
                          n_iters, sched, max_sched);
}
