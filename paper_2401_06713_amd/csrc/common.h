// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>

#include "../../include/picasso.h"

namespace picasso {

// ---- errors ---------------------------------------------------------------
struct Error : std::runtime_error {
    int32_t code;
    Error(int32_t c, const std::string &m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string &msg);

#define PCHECK_HIP(expr)                                                                              \
    do {                                                                                              \
        hipError_t e_ = (expr);                                                                       \
        if (e_ != hipSuccess)                                                                         \
            throw ::picasso::Error(PICASSO_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define PCHECK_LAUNCH() PCHECK_HIP(hipGetLastError())

// ---- constants shared by the kernels --------------------------------------
constexpr uint32_t TAG_LIST = 0x4C495354u;
constexpr uint32_t TAG_PRIO = 0x5052494Fu;
constexpr int32_t COL_UNDECIDED = -2;
constexpr int32_t COL_FAILED = -1;

// ---- XCD-aware workgroup order ---------------------------------------------
// The dispatcher hands workgroups to the eight XCDs in turn (workgroup i to
// XCD i mod 8), and each XCD has an L2 of its own.  For work whose
// neighbouring items share output or input cache lines, this maps workgroup
// ids to items so that each XCD takes one contiguous run of items in order;
// the few items past the last multiple of eight keep their own ids.  A
// bijection on [0, n).
__device__ __forceinline__ int64_t xcd_item(int64_t bid, int64_t n)
{
    const int64_t q = n >> 3;
    if (bid >= (q << 3)) return bid;
    return (bid & 7) * q + (bid >> 3);
}

// ---- Philox4x32-10, device side --------------------------------------------
// Counter (v, s, ell, tag), key (seed lo, seed hi); returns word1:word0.
__device__ __forceinline__ uint64_t philox_draw(uint64_t seed, uint32_t v, uint32_t s, uint32_t ell, uint32_t tag)
{
    uint32_t c0 = v, c1 = s, c2 = ell, c3 = tag;
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    return ((uint64_t)c1 << 32) | c0;
}

// ---- device buffer owned by a handle ---------------------------------------
struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
};

struct Arena {
    size_t live = 0, peak = 0;
    void *ensure(DevBuf &b, size_t bytes);  // grow-only; contents not kept
    void release(DevBuf &b);
};

// ---- a batch of instances during one iteration -----------------------------
// Every kernel works on the concatenation of the active instances of a
// batch; a single instance is a batch of one.  Active vertices of one
// instance are contiguous (compaction keeps their order), each instance's
// palette is a range of one batch-wide colour space, and each bucket holds
// members of a single instance.  The kernels read per-instance values from
// this record and reach it through vinst (per active vertex) or binst (per
// bucket).
// Slot of a list entry (its place in the vertex's sorted list): lists hold
// at most PICASSO_MAX_T colours.
using slot_t = uint16_t;
static_assert(PICASSO_MAX_T <= 65536, "slot_t holds every list position");

struct InstRec {
    int64_t vstart;  // first active vertex of the instance (index into ids)
    int64_t m;       // active vertices
    int64_t loff;    // first list entry of the instance
    int64_t pal;     // first batch-wide colour of the instance's palette
    int64_t P;       // palette size
    int64_t sbase;   // first string of the instance in the packed arrays
    int64_t cbase;   // instance-local id of the palette's first colour (colours of earlier iterations)
    uint64_t seed;
    int32_t T;       // list size
    int32_t rel;     // PICASSO_REL_*
};

struct Batch {
    const InstRec *inst;  // [nb]
    int32_t nb;
    const int32_t *vinst; // [m] instance of each active vertex
    const int64_t *loff;  // [m+1] first list entry of each active vertex; T_v = loff[v+1] - loff[v]
    const int32_t *binst; // [P] instance of each bucket
};

// ---- launch wrappers (each defined in the TU that holds its kernels) ------

// scan.hip: exclusive prefix sums on the device.  `tmp` is scratch of at
// least scan_tmp_bytes(n) bytes.  out[n] receives the total when out has
// room for n+1 entries (with_total).
size_t scan_tmp_bytes(int64_t n);
void exclusive_scan_u32_to_i64(const uint32_t *in, int64_t *out, int64_t n, bool with_total, void *tmp,
                               hipStream_t st);
void exclusive_scan_i32_to_i64(const int32_t *in, int64_t *out, int64_t n, bool with_total, void *tmp,
                               hipStream_t st);

// lists.hip
// Instance and list offset of every active vertex; instance of every bucket.
void launch_vertex_table(const Batch &b, int64_t m, int32_t *vinst, int64_t *loff, hipStream_t st);
void launch_bucket_table(const Batch &b, int64_t P, int32_t *binst, hipStream_t st);
// Lists of every active vertex (batch-wide colours, rows sorted) and the
// priorities; T_max is the largest list size of the batch.
void launch_sample_lists(const Batch &b, uint32_t ell, int64_t m, const int32_t *ids, int32_t T_max,
                         uint32_t *lists, uint64_t *prio, hipStream_t st);
void launch_bucket_count(const uint32_t *lists, int64_t entries, uint32_t *bcnt, hipStream_t st);
void launch_bucket_scatter(const uint32_t *lists, int64_t m, const int64_t *loff, const int64_t *bstart,
                           uint32_t *bfill, uint32_t *bmem, slot_t *bslot, hipStream_t st);
void launch_check_padding(const uint64_t *x, const uint64_t *z, int64_t n, int32_t q, int32_t *bad,
                          hipStream_t st);

// lists.hip: bucket order.  Sorts each bucket's members by (priority,
// local index); pos_of[loff[v] + k] receives the bucket position of (v, k)
// and bent[position] its list entry loff[v] + k (the inverse permutation, so
// that kernels walking a bucket read their members' list entries in order).
void launch_bucket_sort(const int64_t *bstart, int64_t P, uint32_t *bmem, slot_t *bslot, const uint64_t *prio,
                        int64_t *pos_of, int64_t *bent, const int64_t *loff, bool has_large, uint32_t *tmp_mem,
                        slot_t *tmp_slot, hipStream_t st);
// Sum of C(|B_c|, 2) into pairs[0], largest |B_c| into pairs[1].
void launch_bucket_pairs(const uint32_t *bcnt, int64_t P, unsigned long long *pairs, hipStream_t st);
void launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t st);
void launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t st);
void launch_fill_u64(uint64_t *p, int64_t n, uint64_t v, hipStream_t st);
void launch_fill_u8(uint8_t *p, int64_t n, uint8_t v, hipStream_t st);
// Per-bucket words: tiles[c] = ceil(S/64) row tiles, words[c] = S*ceil(S/64).
void launch_bucket_shapes(const int64_t *bstart, int64_t P, int64_t *tiles, int64_t *words, hipStream_t st);
void exclusive_scan_i64(const int64_t *in, int64_t *out, int64_t n, bool with_total, void *tmp, hipStream_t st);

// relate.hip: the relation bit matrices (popcount and int8 MFMA forms).
struct RelateArgs {
    const int64_t *bstart;    // [P+1]
    const uint32_t *bmem;     // local vertex of each bucket entry (priority order)
    int64_t P;
    const int64_t *tile_off;  // [P+1] exclusive scan of ceil(S_c/64)
    int64_t total_row_tiles;
    const int64_t *rb_off;    // [P+1] word offset of each bucket's bit matrix
    const int32_t *ids;       // local -> original id
    const uint64_t *xz;       // all n strings, row i = [x words | z words] (n x 2W)
    int32_t W;
    int32_t relation;         // the relation this launch evaluates
    const int32_t *binst;     // instance of each bucket
    const InstRec *inst;      // buckets whose instance has another relation are skipped
    uint64_t *R;              // relation bit matrices
    const uint64_t *bx, *bz;  // member strings in bucket order (set by launch_relate_prep)
    const int32_t *tile_bucket;  // owner bucket of each row tile (set by launch_relate_prep)
    int64_t mfma_max_members;    // buckets up to this size go to the MFMA kernel (-1: none)
};
// Interleaved copy of the strings: row i = [x_i words | z_i words].
void launch_interleave(const uint64_t *x, const uint64_t *z, int64_t n, int32_t W, uint64_t *xz, hipStream_t st);
// Gathers member strings into bucket order and the row-tile owners.
void launch_relate_prep(RelateArgs &a, int64_t entries, uint64_t *bx, uint64_t *bz, int32_t *tile_bucket,
                        hipStream_t st);
void launch_relate(const RelateArgs &a, hipStream_t st);
// int8 MFMA relation path: whether q and the relation fit it, the largest
// bucket it takes, and the launch (buckets above the cap stay on the VALU
// kernel, which skips the buckets at or below it).
bool mfma_supported(int32_t q, int32_t relation);
int64_t mfma_member_cap(int32_t q, int32_t relation);
void launch_relate_mfma(const RelateArgs &a, int32_t q, hipStream_t st);

// pairs.hip: pairs sharing a smaller colour (dedup) and the CSR.
struct DupArgs {
    const int64_t *bstart;
    const uint32_t *bmem;
    const slot_t *bslot;
    int64_t P;
    const int64_t *rb_off;
    const uint32_t *lists;  // rows sorted, row v at loff[v]
    const int64_t *loff;
    const int64_t *bent;    // list entry loff[v] + k of each bucket member (v, k)
    const int32_t *binst;   // instance of each bucket (its palette start bounds the colours below it)
    const InstRec *inst;
    const uint64_t *R;      // relation matrices (the exact check visits relation pairs only)
    uint64_t *D;            // pairs sharing a smaller colour (zeroed by the caller)
    uint8_t *dflag;         // per bucket entry: 1 if its D row has a bit (zeroed by the caller)
    uint32_t *slow;         // buckets left to the exact per-pair check
    int32_t *n_slow;
};
void launch_dup(const DupArgs &a, hipStream_t st);
void launch_dup_slow(const DupArgs &a, hipStream_t st);  // count of slow buckets read on the device

struct CsrArgs {
    const int64_t *bstart;
    const uint32_t *bmem;
    const slot_t *bslot;
    int64_t P;
    const int64_t *rb_off;
    const uint64_t *R, *D;
    const uint8_t *dflag;    // per bucket entry: its D row has a bit (rows without one read R alone)
    const int64_t *loff;     // list entry of (v, 0)
    // Segment of member (v, s) in v's CSR row, slot-major with stride seg_m:
    // seg[s * seg_m + v] its edge count (count pass), seg_off[s * seg_m + v]
    // its CSR position (fill pass).  Members of one colour hold it at nearby
    // slots, so a bucket's accesses fall in a few slot rows.
    int32_t *seg;
    const int64_t *seg_off;
    int64_t seg_m;
    int32_t *adj;            // fill pass: CSR column indices
    const int32_t *skip;     // fill pass: if non-null and nonzero, write nothing
    int64_t v_lo, v_hi;      // fill pass: only the rows of vertices in [v_lo, v_hi) ...
    int64_t adj_base;        // ... written at adj[CSR position - adj_base]
};
void launch_count(const CsrArgs &a, hipStream_t st);
void launch_fill(const CsrArgs &a, int64_t max_size, hipStream_t st);  // max_size: largest bucket
// From the segment counts (seg, slot-major with stride m): deg[v] = the
// length of v's row; then, with the row pointers, seg_off = each segment's
// CSR position (rowptr[v] plus the counts of v's earlier slots).
void launch_row_lengths(const int32_t *seg, int64_t m, const int64_t *loff, int32_t *deg, hipStream_t st);
void launch_seg_offsets(const int32_t *seg, int64_t m, const int64_t *loff, const int64_t *rowptr, int64_t *seg_off,
                        hipStream_t st);
// flag = (*total > cap): the CSR of *total entries does not fit cap entries.
void launch_csr_guard(const int64_t *total, int64_t cap, int32_t *flag, hipStream_t st);

// color.hip
struct JpArgs {
    int64_t P;
    const int64_t *bstart;
    const uint32_t *bmem;
    const slot_t *bslot;
    const int64_t *rb_off;
    const uint64_t *R;
    const uint32_t *lists;  // rows sorted, row v at loff[v]
    const int64_t *loff;    // [m+1]; T_v = loff[v+1] - loff[v]
    const int64_t *pos_of;  // bucket position of (vertex, slot)
    const InstRec *inst;    // instance table: a bucket's members share its list size and list offsets
    const int32_t *binst;   // [P] instance of each bucket
    int64_t nw_max;         // words per row of the largest bucket
    int32_t fw;             // words per slot mask = ceil(T_max/64)
    int32_t *col;           // batch-wide colour, -1 failed, -2 undecided
    uint64_t *blk, *fre;    // m x fw: slots known blocked / known free
    int32_t *nblk;          // blocked-slot count per vertex
    int32_t packed;         // lists of at most 32 slots: blk[v] holds both masks (blocked in
                            // bits 0-31, free in bits 32-63), fre and nblk are unused
    uint8_t *st;            // per bucket entry: unknown / taken / not taken
    uint8_t *rdy;           // per bucket entry: 1 once the vertex's lower slots are all known blocked
    unsigned long long *wake_at;  // per bucket: idle, busy, or the first position changed since it was last taken
    int32_t *wl[2];         // worklists of buckets: kJpSeg segments of wl_cap entries each
                            // (bucket c in segment c % kJpSeg)
    int64_t wl_cap;         // entries per segment, ceil(P / kJpSeg)
    int32_t *wl_cnt;        // [kJpSlots][kJpRow]: segment lengths entering round k of a batch
                            // in row k, the current lengths in row kJpCountCell
    unsigned long long *progress;  // [kJpSeg * kJpProgStride]: decided vertices, in kJpSeg counters
    unsigned long long *totals;    // [2]: decided vertices and listed buckets after the last batch
    int64_t m;              // vertices to decide
};
constexpr int kJpMaxBatch = 1024;               // rounds per batch, at most
constexpr int kJpCountCell = kJpMaxBatch + 1;   // current list lengths between batches
constexpr int kJpSlots = kJpMaxBatch + 2;
// Appends and progress counts are spread over kJpSeg counters, each on a
// cache line of its own: a single counter takes one atomic per woken
// bucket and per sweep, which serialise at one address.
constexpr int kJpSeg = 64;
constexpr int kJpCntStride = 32;                 // int32 between segment counters (128 bytes)
constexpr int kJpRow = kJpSeg * kJpCntStride;    // int32 per round's row of counters
constexpr int kJpProgStride = 16;                // uint64 between progress counters (128 bytes)
// Every bucket onto worklist 0 (marked waiting): the current lengths sum to P.
void launch_jp_all(const JpArgs &a, hipStream_t st);
// A batch of `rounds` worklist rounds starting from list `cur`: round k
// reads the segments of lengths in row k and appends to the other list,
// counting in row k + 1 (zeroed when the batch begins, so no round resets a
// counter); the batch's final lengths are kept in row kJpCountCell, and the
// batch's end sums the decided vertices and the listed buckets into totals.
void launch_jp_batch_begin(const JpArgs &a, int32_t rounds, hipStream_t st);
void launch_jp_round(const JpArgs &a, int cur, int32_t k, hipStream_t st);
void launch_jp_batch_end(const JpArgs &a, int32_t rounds, hipStream_t st);
// radix.hip: stable LSD radix sort of (key, 32-bit value) pairs by bits
// [bit_lo, bit_hi) in 8- or 9-bit digits; ping-pongs between the two buffer pairs
// and returns 1 if the result is in the alternate pair.  tmp: at least
// radix_tmp_bytes(n) bytes.
size_t radix_tmp_bytes(int64_t n);
template <typename K>
int radix_sort_pairs(K *keys, uint32_t *vals, K *keys_alt, uint32_t *vals_alt, int64_t n, int bit_lo, int bit_hi,
                     void *tmp, hipStream_t st);
// Vertex order by (priority, index): keys hi[v] = the high half of prio[v]
// and values idx[v] = v for radix_sort_pairs over bits [0, 32); then, on the
// sorted keys and values (perm), the runs of equal high halves ordered by
// the whole priority.
void launch_prio_keys(const uint64_t *prio, int64_t m, uint32_t *hi, uint32_t *idx, hipStream_t st);
void launch_prio_ties(const uint32_t *hi, uint32_t *perm, const uint64_t *prio, int64_t m, hipStream_t st);
// List sizes of the vertices in priority order (perm[r]: the vertex at rank r).
void launch_ranked_sizes(const uint32_t *perm, int64_t m, const int64_t *loff, int32_t *tr, hipStream_t st);
// (colour, entry index) of every list entry, vertices in priority order
// (at[r]: first output position of rank r).
void launch_emit_ranked(const uint32_t *perm, int64_t m, const int64_t *loff, const int64_t *at,
                        const uint32_t *lists, uint32_t *keys, uint32_t *vals, int64_t E, hipStream_t st);
// Buckets from the entries sorted by colour (stable from priority order):
// starts, sizes, members, slots, and the position <-> entry maps.
void launch_bucket_from_sorted(const Batch &b, const uint32_t *keys, const uint32_t *ents, int64_t E, int64_t P,
                               int64_t *bstart, uint32_t *bcnt, uint32_t *bmem, slot_t *bslot, int64_t *pos_of,
                               int64_t *bent, hipStream_t st);
constexpr int64_t kRadixMinEntries = (int64_t)1 << 20;  // below: atomics and per-bucket sorts (fewer launches)

// dynamic.hip: the round form of the dynamic-order colouring (Alg. 2).
struct DynArgs {
    Batch b;                      // instances, vinst, loff
    int64_t m, P;
    const int32_t *ids;           // [m] packed string index of each vertex
    const int64_t *pos_of;        // bucket position of (v, k)
    const int64_t *bstart;
    const uint32_t *bmem;
    const slot_t *bslot;
    const int64_t *rb_off;
    const uint64_t *R;            // per-bucket relation rows (symmetric)
    int64_t nw_max;               // words per row of the largest bucket
    int32_t fw;                   // words per slot mask
    uint64_t *alive;              // m x fw: slots still in the list
    int32_t *size;                // [m] slots still in the list
    int32_t *col;                 // [m] batch-wide colour, COL_FAILED, COL_UNDECIDED
    uint64_t *rkey;               // [m] request key: size << 32 | draw
    uint8_t *st;                  // per bucket entry: none / requested / removed
    unsigned long long *hist;     // nb x hist_w: active vertices by list size
    int32_t hist_w;               // largest T + 1
    int32_t *sstar;               // [nb] request threshold: list size
    uint64_t *cut;                // [nb] request threshold: draw
    unsigned long long *active;   // active vertices at the start of the last round
    int32_t divisor;              // about one active vertex in `divisor` requests per round
    uint32_t ell;                 // iteration (keys the draws)
};
void launch_dyn_init(const DynArgs &a, hipStream_t st);
// One round: failures and size counts, thresholds, requests, per-bucket
// resolution and removal.
void launch_dyn_round(const DynArgs &a, int32_t round, hipStream_t st);
void launch_csr_to_relation(int64_t m, const int64_t *rowptr, const int32_t *adj, const uint32_t *lists,
                            const int64_t *loff, const int64_t *pos_of, const int64_t *bstart, const int64_t *rb_off,
                            uint64_t *R, hipStream_t st);
// Output colours (instance-local ids: cbase + colour - pal, written at the
// vertex's packed string index), used-colour counts per instance and the
// uncoloured flags.
void launch_finish_iteration(const Batch &b, int64_t m, const int32_t *col, const int32_t *ids, int32_t *out_colors,
                             uint32_t *used_bits, unsigned long long *n_used, int32_t *uncol_flag, hipStream_t st);
// Per instance: vertices left (from the compaction positions) and conflict
// edges (from the CSR row pointers, halved).
void launch_instance_totals(const Batch &b, const int64_t *pos, const int64_t *rowptr, int64_t *m_next,
                            int64_t *edges, hipStream_t st);
void launch_compact_ids(int64_t m, const int32_t *ids, const int32_t *flag, const int64_t *pos, int32_t *next_ids,
                        hipStream_t st);

// tail.hip: every remaining iteration of an instance with at most kTailMax
// uncoloured vertices, one workgroup per instance.
constexpr int kTailMax = 256;        // vertices
constexpr int kTailListCap = 16384;  // list entries (m x T) of any iteration
struct TailRec {
    int64_t src;    // first vertex id in the ids array
    int64_t m;      // vertices left
    int64_t sbase;  // first packed string of the instance
    int64_t cbase;  // instance-local id of the next palette's first colour
    uint64_t seed;
    int32_t ell;    // number of the next iteration
    int32_t rel;
    int32_t table;  // (P, T) of m vertices at table[table + 2m], table[table + 2m + 1]
    int32_t iter0;  // first slot for the instance's iteration records
};
struct TailOut {
    int64_t n_colors;  // distinct colours used by the tail iterations
    int32_t n_iters;
    int32_t reserved;
};
struct TailIter {
    int64_t m, P, T, pair_tests, edges, colored, offset;
};
void launch_tail(const TailRec *recs, int32_t n, const int32_t *ids, const uint64_t *xz, int32_t W,
                 const int32_t *table, int32_t *out_colors, TailOut *outs, TailIter *iters, hipStream_t st);
// dst[j] for j < total from src ranges: ranges holds nr (src start, dst start)
// pairs, ascending dst starts.
void launch_gather_ranges(const int32_t *src, int32_t *dst, const int64_t *ranges, int32_t nr, int64_t total,
                          hipStream_t st);

// learned.hip: features of the current vertex set and the predictor network.
constexpr int kMlpIn = 6, kMlpHidden = 64, kMlpOut = 2;
constexpr int kMlpParams = kMlpHidden * kMlpIn + kMlpHidden + kMlpHidden * kMlpHidden + kMlpHidden +
                           kMlpOut * kMlpHidden + kMlpOut;
constexpr int kMlpKeep = kMlpIn + 2 * kMlpHidden + kMlpOut + 2 * kMlpHidden;  // per-row training state
constexpr int kFeaturePairs = 4096;
constexpr int kSizingPairs = 16384;  // sampled pairs of the CSR size bound (the first 4096 are the features')
void launch_features(int64_t m, const int32_t *ids, const uint64_t *x, const uint64_t *z, int32_t W, uint64_t seed,
                     uint32_t ell, int32_t rel, int32_t K, unsigned long long *weight, unsigned long long *hits,
                     hipStream_t st);
// Relation density of every instance of a batch: hits[a] (zeroed by the
// caller) counts the K sampled pairs of the instance's active vertices that
// the relation joins -- the pairs the features kernel samples, keyed by the
// instance's seed.
void launch_density(const Batch &b, const int32_t *ids, const uint64_t *x, const uint64_t *z, int32_t W, uint32_t ell,
                    int32_t K, uint32_t *hits, hipStream_t st);
// Forward pass over B rows (out: B x 2 raw outputs, may be null); with
// target/keep/row_loss non-null it also stores the training state.
void launch_mlp_rows(const float *p, const float *raw, int32_t B, float *out, const float *target, float *keep,
                     float *row_loss, hipStream_t st);
void launch_mlp_grad(const float *keep, int32_t B, float *grad, hipStream_t st);
void launch_adam(float *p, const float *g, float *m1, float *m2, float lr, float b1, float b2, float eps, int32_t step,
                 hipStream_t st);
void launch_squash(const float *o, int32_t B, float *fa, hipStream_t st);

}  // namespace picasso
