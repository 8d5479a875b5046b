/*
 * picasso.h -- C ABI of the MI355X palette-colouring library (libpicasso.so).
 *
 * The library groups Pauli strings by colouring the graph whose edges are
 * the pairs that FAIL the grouping relation, with the palette-sparsification
 * method of Picasso (arXiv 2401.06713): each iteration draws a random colour
 * list per vertex (Alg. 1, assign_rand_list_colors), builds the conflict
 * graph of relation edges whose endpoints share a list colour (Alg. 1
 * construct_conflict_graph; Sec. IV-A), list-colours it in a random static
 * order (Sec. IV-B, static order schemes) and recurses on the uncoloured
 * vertices with a fresh palette (Alg. 1).  A colour class is therefore a set
 * of mutually commuting (ANTICOMMUTE relation) or qubit-wise commuting (QWC
 * relation) strings.
 *
 * Conventions shared by every entry point:
 *  - A Pauli string on q qubits is two bit-planes x and z of W = ceil(q/64)
 *    uint64 words; qubit k is bit k%64 of word k/64; (x,z) = (0,0) I,
 *    (1,0) X, (1,1) Y, (0,1) Z.  Arrays of n strings are row-major n x W.
 *    Bits >= q of the last word must be zero.
 *  - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *    device memory of the current device (e.g. a torch tensor's data_ptr).
 *  - Every call returns a negative PICASSO_E* code on failure and records a
 *    message readable with picasso_last_error() on the same thread; no C++
 *    exception crosses this boundary.
 *  - A handle is not thread-safe: use one handle per host thread.  All work
 *    of a handle runs on its stream; calls return after that stream has
 *    finished the work unless stated otherwise.
 */
#ifndef PICASSO_H
#define PICASSO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct picasso_ctx *picasso_handle;

/* Grouping relations: an edge joins two strings that fail the relation. */
enum {
    PICASSO_REL_ANTICOMMUTE = 0, /* edge iff the strings anticommute: odd number of
                                    anticommuting positions (Sec. IV-A, Eq. 5)      */
    PICASSO_REL_QWC = 1,         /* edge iff not qubit-wise commuting: some position
                                    holds two different non-identity Paulis (Sec. III) */
    PICASSO_REL_COMMUTE = 2      /* edge iff the strings commute: even number of
                                    anticommuting positions.  The orientation of the
                                    paper's unitary-partitioning application (Sec. II,
                                    Sec. IV-A): colour classes are sets of mutually
                                    anticommuting strings.  Identical strings commute,
                                    so duplicates always conflict.                     */
};

/* Return codes. */
enum {
    PICASSO_OK = 0,
    PICASSO_EINVAL = -1,   /* bad argument; nothing was changed                */
    PICASSO_ENOMEM = -2,   /* a device allocation failed, or one row of the
                              CSR asked of picasso_conflict_graph exceeds the
                              memory budget                                   */
    PICASSO_EDEVICE = -3,  /* a HIP call failed; the message names it           */
    PICASSO_EINTERNAL = -4 /* internal invariant violated                        */
};

/* Options for picasso_set_option. */
enum {
    PICASSO_OPT_MEM_BUDGET = 1, /* max device bytes for one iteration's conflict
                                   graph (CSR); 0 = no limit beyond the device.
                                   Above it picasso_conflict_graph writes the
                                   CSR in chunks of whole rows of at most this
                                   many bytes (ENOMEM if one row exceeds it);
                                   the colouring calls count the edges and
                                   skip writing the CSR (they colour from the
                                   per-bucket relation matrices)                */
    PICASSO_OPT_PAIR_PATH = 2,  /* 0 auto (= 1: the popcount kernel measured
                                   faster on every workload), 1 popcount VALU,
                                   2 int8 MFMA (EINVAL where q and the relation
                                   do not fit its LDS rows)                   */
    PICASSO_OPT_FIXED_T = 3,    /* >0: list size T fixed (clamped to P) instead of
                                   ceil(alpha ln m); 0 restores the formula      */
    PICASSO_OPT_STREAM = 4,     /* hipStream_t (cast to int64) to run on; 0 = the
                                   handle's own stream.  The caller keeps the
                                   stream alive while the handle uses it.        */
    PICASSO_OPT_TIMING = 5,     /* 1: record per-phase times (adds event syncs)  */
    PICASSO_OPT_JP_BATCH = 6,   /* colouring rounds launched between two host
                                   checks of progress, at most (1..1024; 32)    */
    PICASSO_OPT_GRAPH = 7,      /* 1 (default): a full batch of colouring rounds
                                   is captured once per iteration into a HIP
                                   graph and replayed; 0: plain launches        */
    PICASSO_OPT_MFMA_CAP = 8,   /* MFMA pair path: buckets of at most this many
                                   members take the MFMA kernel, larger ones the
                                   popcount tile kernel; -1 (default) = as many
                                   as the kernel's LDS rows hold for this q      */
    PICASSO_OPT_TAIL = 9,       /* 1 (default): an instance with at most 256
                                   vertices left (and lists within the kernel's
                                   LDS) finishes its iterations in one device
                                   workgroup; 0: every iteration takes the full
                                   path.  Results are identical.  Iterations
                                   run there report pair_path 0 and no times.  */
    PICASSO_OPT_LEARNED_JUDGE = 10, /* picasso_color_learned: 1 = also colour with
                                   the fixed parameters (f = 0.125, alpha = 2)
                                   and return whichever result has fewer
                                   colours (the network's on a tie); stats
                                   record which (picasso_stats.judged) and the
                                   time of both runs.  0 (default): the
                                   network's result only.                     */
    PICASSO_OPT_CSR_SIZING = 11, /* colouring calls: 1 (default) = each iteration's
                                   CSR buffer is sized by the predicted bound on
                                   |E_c| (picasso_iter_stats.edges_bound) and
                                   filled without waiting for the exact size;
                                   an iteration above the bound is filled again
                                   at its exact size (picasso_stats.csr_refills).
                                   0 = the exact size is read back before the
                                   fill.  2 = the bound taken as zero, so every
                                   iteration refills (tests that path).
                                   Results are identical.                     */
    PICASSO_OPT_COLOURER = 12,  /* list colouring of each iteration:
                                   PICASSO_COLOURER_STATIC (default) or
                                   PICASSO_COLOURER_DYNAMIC                   */
    PICASSO_OPT_DYN_DIVISOR = 13, /* dynamic colourer: about one active vertex in
                                   this many requests a colour per round
                                   (1..2^20; 16).  Larger: closer to the
                                   sequential order, more rounds.             */
    PICASSO_OPT_BUCKET_BUILD = 15, /* colour buckets: 0 (default) auto, 1 = an
                                   atomic count and scatter per list entry,
                                   then a sort of each bucket by priority;
                                   2 = a stable radix sort (vertices by
                                   priority, then their entries by colour).
                                   Auto takes the radix sort from 2^20 list
                                   entries.  Results are identical.           */
    PICASSO_OPT_EDGES = 14      /* colouring calls: 1 (default) = each iteration
                                   also counts its conflict edges and writes its
                                   CSR (min-shared-colour dedup, counts, fill);
                                   0 = only the per-bucket relation matrices the
                                   colouring reads are built, and the edge
                                   statistics of those iterations are -1.  The
                                   colours are identical.  For long lists over
                                   small palettes (buckets of thousands of
                                   members, e.g. palette 3%, alpha 30) the dedup
                                   dominates the run time.                    */
};

/* Colourers (PICASSO_OPT_COLOURER). */
#define PICASSO_COLOURER_STATIC 0  /* random static order, smallest free list
                                      colour (Sec. IV-B, static order schemes):
                                      equals the sequential greedy in
                                      (priority, id) order                    */
#define PICASSO_COLOURER_DYNAMIC 1 /* dynamic order, Alg. 2 (Sec. IV-B): the
                                      shortest remaining lists first, a random
                                      colour of the list, the colour removed
                                      from the neighbours' lists; run in rounds
                                      in which about one active vertex in
                                      PICASSO_OPT_DYN_DIVISOR (those with the
                                      shortest lists) requests a colour, each
                                      colour's requesters settled in (size,
                                      draw, vertex) order.  Deterministic for a
                                      seed; not the sequential Alg. 2 order.
                                      Instances do not use the tail kernel.   */

/* picasso_stats.judged */
#define PICASSO_JUDGE_NONE 0    /* no judge run                               */
#define PICASSO_JUDGE_LEARNED 1 /* the network's colouring was kept          */
#define PICASSO_JUDGE_FIXED 2   /* the fixed-parameter colouring was kept    */

#define PICASSO_PATH_AUTO 0
#define PICASSO_PATH_VALU 1
#define PICASSO_PATH_MFMA 2

#define PICASSO_MAX_T 1024         /* largest list size the kernels accept   */
#define PICASSO_MAX_ITER_STATS 256 /* per-iteration records kept in stats    */

/* Per-iteration record. Times are milliseconds (0 unless PICASSO_OPT_TIMING). */
typedef struct {
    int64_t m;          /* uncoloured vertices entering the iteration         */
    int64_t P;          /* palette size                                       */
    int64_t T;          /* list size                                          */
    int64_t pair_tests; /* sum over colours c of C(|B_c|, 2)                   */
    int64_t edges;      /* |E_c|, undirected conflict edges (-1: not counted,
                           PICASSO_OPT_EDGES = 0)                             */
    int64_t edges_bound; /* upper bound on |E_c| predicted before the pair pass
                           from the sampled relation density (sizes the CSR;
                           iterations run in the tail kernel count |E_c|
                           exactly and report it here)                       */
    int64_t colored;    /* vertices coloured in this iteration                 */
    int64_t offset;     /* first global colour id of this iteration's palette
                           (single-instance handles; 0 for batches)           */
    int32_t pair_path;  /* PICASSO_PATH_VALU or PICASSO_PATH_MFMA (0: the tail
                           kernel, see PICASSO_OPT_TAIL)                        */
    int32_t jp_rounds;  /* colouring rounds                                    */
    double ms_graph;   /* conflict-graph build: pair pass through CSR fill   */
    double ms_buckets; /* list sampling and colour-bucket build              */
    double ms_count;   /* pair pass (relation bit matrices)                  */
    double ms_fill;    /* CSR fill (edge compaction)                          */
    double ms_color;   /* list colouring rounds                               */
    double ms_compact; /* output colours, counts and the next vertex set      */
} picasso_iter_stats;

/* Summary of the handle's last colouring call. */
typedef struct {
    int64_t n;
    int64_t n_colors;      /* distinct colours used                            */
    int64_t palette_total; /* sum of palette sizes (an upper bound)           */
    int64_t pair_tests;    /* over all iterations                              */
    int64_t edges;         /* over all iterations                              */
    int64_t max_edges;     /* largest single-iteration |E_c|                   */
    int64_t peak_device_bytes;
    int32_t n_iters;
    int32_t judged;  /* PICASSO_JUDGE_* (picasso_color_learned)           */
    int32_t csr_refills; /* iterations whose |E_c| exceeded the predicted bound
                            (their CSR was written again at the exact size) */
    int32_t reserved;
    double ms_total; /* wall time of the call                                */
    picasso_iter_stats iters[PICASSO_MAX_ITER_STATS];
} picasso_stats;

/* Per-instance summary of the last colouring call (for batches, one per
 * instance in creation order; a single-instance handle has one). */
typedef struct {
    int64_t n;             /* strings of the instance                          */
    int64_t n_colors;      /* distinct colours used                            */
    int64_t palette_total; /* sum of its palette sizes                         */
    int64_t edges;         /* conflict edges over all its iterations           */
    int64_t max_edges;     /* largest single-iteration |E_c| of the instance   */
    int32_t n_iters;       /* iterations the instance took                     */
    int32_t reserved;
} picasso_instance_stats;

/* Most recent error message of this host thread ("" if none). */
const char *picasso_last_error(void);

/* Create a handle holding a device copy of n strings on q qubits.
 * x_words, z_words: host, n*W uint64 each (copied; the caller may free them).
 * 0 <= n < 2^31, 1 <= q <= 256.  Duplicate strings are allowed (they are
 * never joined by an edge).  Returns NULL on error (see picasso_last_error):
 * bad sizes, NULL pointers with n > 0, or padding bits set. */
picasso_handle picasso_create(int64_t n, int32_t q, const uint64_t *x_words, const uint64_t *z_words);

/* As picasso_create, but x_words/z_words are device pointers (copied
 * device-to-device; padding bits are checked on the device). */
picasso_handle picasso_create_device(int64_t n, int32_t q, const uint64_t *x_words, const uint64_t *z_words);

/* Create one handle holding `count` independent instances (a batch),
 * coloured together by picasso_color_batch.  Instance i has ns[i] strings on
 * qs[i] qubits (W_i = ceil(qs[i]/64) words); x_words/z_words (host) hold the
 * instances back to back: instance i's n_i x W_i rows follow instance
 * i-1's.  Same limits as picasso_create for every instance, and the total
 * number of strings is below 2^31.  Returns NULL on error. */
picasso_handle picasso_create_batch(int32_t count, const int64_t *ns, const int32_t *qs, const uint64_t *x_words,
                                    const uint64_t *z_words);

/* Release the handle and all device memory it owns.  NULL is ignored. */
void picasso_destroy(picasso_handle h);

/* Set an option (PICASSO_OPT_*).  Returns PICASSO_OK or PICASSO_EINVAL. */
int32_t picasso_set_option(picasso_handle h, int32_t key, int64_t value);

/* Colour all strings (Alg. 1).
 * seed: keys every random draw (lists and priorities).
 * palette_frac f in (0, 1]: iteration palette P = max(1, ceil(f m)).
 * list_size alpha > 0 (a multiplier): T = clamp(ceil(alpha ln m), 1, P).
 * relation: PICASSO_REL_*.
 * out_colors: host, n int32, receives global colour ids (iteration l uses
 * ids [offset_l, offset_l + P_l), offsets cumulative).
 * Returns the number of distinct colours (>= 0) or a negative error. */
int64_t picasso_color(picasso_handle h, uint64_t seed, double palette_frac, double list_size, int32_t relation,
                      int32_t *out_colors);

/* As picasso_color, but out_colors is a device pointer (n int32).  The
 * result is complete when the call returns. */
int64_t picasso_color_device(picasso_handle h, uint64_t seed, double palette_frac, double list_size,
                             int32_t relation, int32_t *out_colors);

/* Colour every instance of a batch handle, each exactly as picasso_color
 * would colour it alone with its own arguments (Alg. 1 per instance; the
 * instances advance through their iterations side by side, each kernel
 * launch covering all instances still holding uncoloured strings).
 * seeds, palette_fracs, list_sizes, relations: host arrays of one entry per
 * instance, meanings as in picasso_color.  out_colors: host int32, the
 * total number of strings, instance i's colours (its own ids from 0) at its
 * strings' positions in the concatenation.  out_n_colors: host int64 per
 * instance.  Returns the sum of the instances' colour counts or an error.
 * The single-instance calls below (picasso_color, picasso_color_device,
 * picasso_sample_lists, picasso_conflict_graph, picasso_list_color_csr,
 * picasso_features, picasso_color_learned) reject batch handles of more
 * than one instance with PICASSO_EINVAL. */
int64_t picasso_color_batch(picasso_handle h, const uint64_t *seeds, const double *palette_fracs,
                            const double *list_sizes, const int32_t *relations, int32_t *out_colors,
                            int64_t *out_n_colors);

/* As picasso_color_batch, but out_colors is a device pointer (int32, the
 * total number of strings); out_n_colors stays on the host.  The result is
 * complete when the call returns. */
int64_t picasso_color_batch_device(picasso_handle h, const uint64_t *seeds, const double *palette_fracs,
                                   const double *list_sizes, const int32_t *relations, int32_t *out_colors,
                                   int64_t *out_n_colors);

/* Copy the last colouring call's statistics (for a batch: iterations
 * aggregated over the instances: m, P, pair_tests, edges, colored summed,
 * T the largest list size).  Returns PICASSO_OK. */
int32_t picasso_get_stats(picasso_handle h, picasso_stats *out);

/* Copy the first `count` per-instance summaries of the last colouring call
 * into out (host).  count = 0 with out = NULL only queries.  Returns the
 * handle's number of instances or an error. */
int32_t picasso_get_instance_stats(picasso_handle h, int32_t count, picasso_instance_stats *out);

/* ---- Single steps of one iteration, for tests and tools ---------------- */

/* Colour lists and priorities of iteration `ell` for the vertices ids[0..m)
 * (host, ascending original ids) with palette P and list size T
 * (1 <= T <= min(P, PICASSO_MAX_T)).  out_lists: host, m*T uint32,
 * row-major, each row sorted ascending (Floyd's sample of a uniform
 * T-subset of [0,P), one Philox4x32-10 draw per step keyed by
 * (seed; vertex, slot, ell)).  out_prio: host, m uint64 (may be NULL). */
int32_t picasso_sample_lists(picasso_handle h, uint64_t seed, int32_t ell, int64_t m, const int32_t *ids,
                             int64_t P, int32_t T, uint32_t *out_lists, uint64_t *out_prio);

/* Conflict graph of iteration `ell` over ids[0..m) (host, ascending):
 * {a, b} is an edge iff the relation holds and the lists share a colour
 * (Alg. 1 construct_conflict_graph; Sec. IV-A).  Output is the symmetric
 * CSR in local indices: out_rowptr host int64[m+1]; out_adj host int32,
 * capacity adj_cap entries (2|E_c| are needed; rows are unordered).  Either
 * output may be NULL to only count.  Returns |E_c| (undirected) or an error;
 * if 2|E_c| > adj_cap nothing is written to out_adj.  When the CSR exceeds
 * PICASSO_OPT_MEM_BUDGET it is filled and copied out in chunks of whole rows
 * (Alg. 3 builds it on the host past the device's memory; here the device
 * writes each chunk within the budget), with the same result. */
int64_t picasso_conflict_graph(picasso_handle h, uint64_t seed, int32_t ell, int64_t m, const int32_t *ids,
                               int64_t P, int32_t T, int32_t relation, int64_t *out_rowptr, int32_t *out_adj,
                               int64_t adj_cap);

/* List-colour a given conflict graph in the random static order: vertices
 * taken by ascending (prio, index), each gets the smallest colour of its
 * list held by no earlier neighbour, or -1 (Sec. IV-B).  Computed in
 * parallel (Jones-Plassmann rounds) with the sequential result.
 * prio host uint64[m]; lists host uint32[m*T] (rows sorted, values < P);
 * rowptr host int64[m+1]; adj host int32[rowptr[m]] (symmetric CSR);
 * out_col host int32[m].  Returns the number of coloured vertices. */
int64_t picasso_list_color_csr(picasso_handle h, int64_t m, const uint64_t *prio, const uint32_t *lists, int32_t T,
                               int64_t P, const int64_t *rowptr, const int32_t *adj, int32_t *out_col);

/* ---- Learned parameters (the paper's Sec. VI predictor, as a small MLP) --- */

typedef struct picasso_mlp_ctx *picasso_mlp;

#define PICASSO_MLP_NPARAMS 4738 /* W1[64][6] b1[64] W2[64][64] b2[64] W3[2][64] b3[2] */
#define PICASSO_MLP_INPUTS 6      /* five features (picasso_features) and beta          */
#define PICASSO_FEATURE_PAIRS 4096

/* Features of an iteration's vertex set: out[5] = (ln m, q, mean Pauli
 * weight, fraction of PICASSO_FEATURE_PAIRS sampled vertex pairs joined by
 * the relation, ell).  ids host, m ascending original ids.  Sampled pair k
 * is keyed by (seed; k, ell).  Returns PICASSO_OK or an error. */
int32_t picasso_features(picasso_handle h, uint64_t seed, int32_t ell, int64_t m, const int32_t *ids,
                         int32_t relation, double *out);

/* A 6 -> 64 -> 64 -> 2 perceptron (ReLU hidden layers, FP32) whose inputs are an iteration's five features and the trade-off weight
 * beta of the bi-objective beta * colours + (1 - beta) * |E_c| (Sec. VI,
 * Eq. 7: the regressor predicts (P', alpha) for a given graph and beta), on
 * the device of the calling thread.  params: host, PICASSO_MLP_NPARAMS floats in the
 * layout above, or NULL for a deterministic initialisation from seed
 * (scaled normal weights, zero biases).  Returns NULL on error. */
picasso_mlp picasso_mlp_create(const float *params, uint64_t seed);
void picasso_mlp_destroy(picasso_mlp mlp);
int32_t picasso_mlp_get_params(picasso_mlp mlp, float *out);      /* host, NPARAMS floats */
int32_t picasso_mlp_set_params(picasso_mlp mlp, const float *in);  /* resets the Adam state */

/* Raw outputs o (B x 2, host) for B input rows (B x 6, host: the five
 * features of picasso_features, then beta); the
 * parameters are f = 0.01 + 0.24 sigmoid(o0), alpha = 1 + 3 sigmoid(o1). */
int32_t picasso_mlp_forward(picasso_mlp mlp, const float *features, int32_t B, float *out);

/* Loss (1/(2B)) sum (o - target)^2 over B rows and its gradient (host,
 * NPARAMS floats; may be NULL).  Returns PICASSO_OK. */
int32_t picasso_mlp_gradient(picasso_mlp mlp, const float *features, const float *target, int32_t B, float *grad,
                             float *loss);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on a batch; writes the
 * batch loss before the step to *loss.  Returns PICASSO_OK. */
int32_t picasso_mlp_train_step(picasso_mlp mlp, const float *features, const float *target, int32_t B, float lr,
                               float *loss);

/* Colour with per-iteration parameters from the network: each iteration
 * computes its features on the device, runs the network on them and beta
 * (in [0, 1], the weight of the colour count in Eq. 7), and uses the FP32
 * (f, alpha) it returns (Sec. VI: parameters predicted from the graph and
 * beta).  Fallback: an iteration whose outputs are not finite or fall
 * outside f in (0, 1], alpha > 0 uses the fixed parameters f = 0.125,
 * alpha = 2 (the paper's evaluation default).  Judge: with
 * PICASSO_OPT_LEARNED_JUDGE = 1 the fixed-parameter colouring runs as well
 * and the result with fewer colours is returned.  out_schedule (host,
 * 2 * max_sched floats, may be NULL) receives the network's (f, alpha) of
 * the first max_sched iterations.  Returns n_colors or an error. */
/* Colour with an explicit schedule of parameters (Alg. 1 with the
 * per-iteration palette and list size chosen by the caller, as the learned
 * predictor of Sec. VI chooses them): iteration l (from 1) uses
 * palette_fracs[k] and list_sizes[k] with k = min(l, count) - 1, so the last
 * entry repeats.  palette_fracs, list_sizes: host, count >= 1 entries, each
 * valid as in picasso_color.  Output and errors as picasso_color. */
int64_t picasso_color_schedule(picasso_handle h, uint64_t seed, const double *palette_fracs, const double *list_sizes,
                               int32_t count, int32_t relation, int32_t *out_colors);

int64_t picasso_color_learned(picasso_handle h, uint64_t seed, picasso_mlp mlp, double beta, int32_t relation,
                              int32_t *out_colors, float *out_schedule, int32_t max_sched);

/* ---- Colouring without device allocation ------------------------------- */

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): the same colouring as
 * picasso_color_device on a handle created from these strings, for at most
 * PICASSO_NOALLOC_MAX_N strings, with no handle and no allocation.  Every
 * iteration runs in one device workgroup; its working memory (staged
 * strings, the (P, T) table, iteration records, a padding flag) is a fixed
 * PICASSO_NOALLOC_SCRATCH_BYTES array that each device holds from the first
 * call until the process ends.
 * x_words, z_words: device, n*W uint64 each (W = ceil(q/64)), padding bits
 * zero; out_colors: device, n int32 (global colour ids as from
 * picasso_color_device); seed, palette_frac, list_size, relation: as in
 * picasso_color; stream: hipStream_t to run on (NULL: the null stream).
 * Returns the number of distinct colours, or PICASSO_EINVAL when
 * n > PICASSO_NOALLOC_MAX_N, when some iteration's lists would exceed
 * PICASSO_NOALLOC_MAX_LIST_ENTRIES entries (T x m), or on the argument
 * errors of picasso_create / picasso_color.  Calls on one device share its
 * array: calls that overlap on one device (other threads, other streams)
 * race and must be serialised by the caller.  Returns after the stream has
 * finished the work. */
#define PICASSO_NOALLOC_MAX_N 256
#define PICASSO_NOALLOC_MAX_LIST_ENTRIES 16384
#define PICASSO_NOALLOC_SCRATCH_BYTES 65536
int64_t picasso_color_device_noalloc(int64_t n, int32_t q, const uint64_t *x_words, const uint64_t *z_words,
                                     uint64_t seed, double palette_frac, double list_size, int32_t relation,
                                     int32_t *out_colors, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* PICASSO_H */
