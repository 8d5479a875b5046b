// Host driver and C ABI (Alg. 1 iteration loop around the device steps).
//
// Per iteration: (P, T) in host double arithmetic -> lists and priorities ->
// colour buckets (count, scan, scatter) -> pair count pass -> row-pointer
// scan -> pair fill pass into the CSR -> list colouring -> write global
// colours, compact the uncoloured vertices (ascending ids) -> next palette.
// The only device->host traffic inside the loop is a few scalars.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <random>
#include <vector>

#include "common.h"

namespace picasso {

static thread_local std::string g_last_error;
void set_last_error(const std::string &msg) { g_last_error = msg; }

void *Arena::ensure(DevBuf &b, size_t bytes)
{
    if (bytes == 0) bytes = 1;
    if (b.cap >= bytes) return b.p;
    if (b.p) {
        PCHECK_HIP(hipFree(b.p));
        live -= b.cap;
        b.p = nullptr;
        b.cap = 0;
    }
    const size_t want = bytes + bytes / 8;  // headroom for the next iteration's growth
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        e = hipMalloc(&b.p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            b.p = nullptr;
            throw Error(PICASSO_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
        }
        b.cap = bytes;
    } else {
        b.cap = want;
    }
    live += b.cap;
    if (live > peak) peak = live;
    return b.p;
}

void Arena::release(DevBuf &b)
{
    if (b.p) {
        (void)hipFree(b.p);
        live -= b.cap;
    }
    b.p = nullptr;
    b.cap = 0;
}

}  // namespace picasso

using namespace picasso;

struct picasso_ctx {
    int64_t n = 0;           // strings over all instances
    int32_t q = 0, W = 0;    // largest q of the instances; words per packed string
    int32_t nb = 1;          // instances
    std::vector<int64_t> inst_n, inst_base;  // strings of each instance, first packed string
    std::vector<int32_t> inst_q;
    int device = 0;
    hipStream_t own_stream = nullptr;
    hipStream_t tail_stream = nullptr;  // tail kernels, beside the main path (created on first use)
    hipEvent_t tail_ready = nullptr, tail_done = nullptr;
    hipStream_t stream = nullptr;
    int64_t mem_budget = 0;
    int32_t pair_path = PICASSO_PATH_AUTO;
    int32_t fixed_T = 0;
    int32_t timing = 0;
    int32_t jp_batch = 32;   // colouring rounds per host check, at most
    int32_t use_graph = 1;   // replay colouring rounds from a captured graph
    int64_t mfma_cap = -1;   // largest bucket for the MFMA kernel (-1: as large as LDS allows)
    int32_t use_tail = 1;    // finish instances with few vertices left in the tail kernel
    int32_t judge = 0;       // learned colouring: also run the fixed parameters, keep the better
    int32_t edges_on = 1;    // colouring calls: count the conflict edges and write the CSR
    int32_t bucket_build = 0;  // 0 auto, 1 atomics + per-bucket sort, 2 radix sort
    int32_t colourer = PICASSO_COLOURER_STATIC;
    int32_t dyn_divisor = 16;  // dynamic colourer: about one active vertex in this many requests per round
    int64_t seg_m = 0;       // vertex stride of h->seg (the last conflict-graph build's m)
    int32_t csr_sizing = 1;  // colouring calls: 1 CSR sized by the predicted bound, 0 by the exact
                             // size, 2 bound forced to zero (every iteration refills; for tests)
    Arena arena;
    DevBuf x, z, xz;  // bit-planes, and the interleaved copy the member gather reads
    // iteration buffers
    DevBuf ids, next_ids, lists, prio, bcnt, bstart, bmem, bslot, pos_of, bent, tmp_mem, tmp_slot, tiles, words, tile_off,
        rb_off, R, D, bx, bz, tile_bucket, nslow, slow, seg, seg_off, deg, rowptr, adj, col, blk, fre, nblk, st, rdy, jp_prog, dflag,
        wake_at, wl, flags, pos, used, scan_tmp, scalars, out_colors, judge_out, inst, vinst, loff, binst,
        inst_out, tail_recs, tail_table, tail_outs, tail_iters, tail_ranges, tail_ids, hits, csr_flag, rkey, dyn_hist, dyn_sstar,
        dyn_cut, rx_k32a, rx_k32b, rx_va, rx_vb, rx_tmp, rx_tr, rx_at, rx_cka, rx_ckb, rx_cva, rx_cvb;
    std::vector<InstRec> h_inst;  // table of the active instances (kept until the copy has completed)
    picasso_stats stats;
    std::vector<picasso_instance_stats> istats;
};

struct picasso_mlp_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    Arena arena;
    DevBuf params, m1, m2, raw, target, out, keep, row_loss, grad, fa;
    int32_t step = 0;
};

namespace {

// The fixed parameters of the paper's evaluation (palette 12.5% of the
// vertices, alpha = 2): the learned colouring's fallback and judge.
constexpr double kFixedFrac = 0.125, kFixedAlpha = 2.0;

template <typename T>
T *mbuf(picasso_mlp_ctx *c, DevBuf &b, size_t count)
{
    return static_cast<T *>(c->arena.ensure(b, count * sizeof(T)));
}

template <typename T>
T *buf(picasso_ctx *h, DevBuf &b, size_t count)
{
    return static_cast<T *>(h->arena.ensure(b, count * sizeof(T)));
}

void params(int64_t m, double frac, double alpha, int32_t fixed_T, int64_t &P, int32_t &T)
{
    const double pd = std::ceil(frac * (double)m);
    P = (int64_t)pd;
    if (P < 1) P = 1;
    int64_t t = fixed_T > 0 ? fixed_T : (int64_t)std::ceil(alpha * std::log((double)m));
    if (t < 1) t = 1;
    if (t > P) t = P;
    T = (int32_t)t;
}

struct Timer {
    picasso_ctx *h;
    hipEvent_t ev[8];
    int k = 0;
    explicit Timer(picasso_ctx *hh) : h(hh)
    {
        if (h->timing)
            for (auto &e : ev) PCHECK_HIP(hipEventCreate(&e));
    }
    ~Timer()
    {
        if (h->timing)
            for (auto &e : ev) (void)hipEventDestroy(e);
    }
    void mark()
    {
        if (h->timing && k < 8) PCHECK_HIP(hipEventRecord(ev[k++], h->stream));
    }
    double ms(int a, int b)
    {
        if (!h->timing || b >= k) return 0.0;
        PCHECK_HIP(hipEventSynchronize(ev[b]));
        float f = 0.f;
        PCHECK_HIP(hipEventElapsedTime(&f, ev[a], ev[b]));
        return f;
    }
};

template <typename T>
T read_scalar(picasso_ctx *h, const T *dptr)
{
    T v;
    PCHECK_HIP(hipMemcpyAsync(&v, dptr, sizeof(T), hipMemcpyDeviceToHost, h->stream));
    PCHECK_HIP(hipStreamSynchronize(h->stream));
    return v;
}

void upload(picasso_ctx *h, void *dst, const void *src, size_t bytes)
{
    if (bytes) PCHECK_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, h->stream));
}

void download(picasso_ctx *h, void *dst, const void *src, size_t bytes)
{
    if (bytes) PCHECK_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, h->stream));
    PCHECK_HIP(hipStreamSynchronize(h->stream));
}

// Uploads h->h_inst (the active instances, vstart/loff/pal ascending) and
// derives the per-vertex table for the m active vertices.
Batch upload_batch(picasso_ctx *h, int64_t m)
{
    const size_t nb = h->h_inst.size();
    InstRec *d = buf<InstRec>(h, h->inst, nb);
    upload(h, d, h->h_inst.data(), nb * sizeof(InstRec));
    Batch b{};
    b.inst = d;
    b.nb = (int32_t)nb;
    int32_t *vinst = buf<int32_t>(h, h->vinst, (size_t)std::max<int64_t>(m, 1));
    int64_t *loff = buf<int64_t>(h, h->loff, (size_t)m + 1);
    launch_vertex_table(b, m, vinst, loff, h->stream);
    b.vinst = vinst;
    b.loff = loff;
    return b;
}

// A table of one instance over the m given vertices (ids in h->ids).
Batch single_instance(picasso_ctx *h, uint64_t seed, int64_t m, int64_t P, int32_t T, int32_t rel)
{
    InstRec r{};
    r.vstart = 0;
    r.m = m;
    r.loff = 0;
    r.pal = 0;
    r.P = P;
    r.sbase = 0;
    r.cbase = 0;
    r.seed = seed;
    r.T = T;
    r.rel = rel;
    h->h_inst.assign(1, r);
    return upload_batch(h, m);
}

struct BucketInfo {
    int64_t pair_tests = 0;  // sum over colours of C(|B_c|, 2)
    int64_t max_size = 0;    // largest bucket
    int64_t row_tiles = 0;   // sum of ceil(|B_c|/64)
    int64_t words = 0;       // sum of |B_c| * ceil(|B_c|/64)
};

// Buckets of the lists already in h->lists (E entries over the m vertices
// of batch b, P colours): count, scan, scatter, sort by priority (h->prio),
// the shapes of the per-bucket bit matrices and the bucket -> instance
// table (b.binst is set).
BucketInfo buckets_from_lists(picasso_ctx *h, Batch &b, int64_t m, int64_t E, int64_t P,
                              const uint32_t *d_hits = nullptr, uint32_t *h_hits = nullptr)
{
    hipStream_t st = h->stream;
    const uint32_t *lists = static_cast<const uint32_t *>(h->lists.p);
    const uint64_t *prio = static_cast<const uint64_t *>(h->prio.p);
    uint32_t *bcnt = buf<uint32_t>(h, h->bcnt, (size_t)P);
    int64_t *bstart = buf<int64_t>(h, h->bstart, (size_t)P + 1);
    unsigned long long *sc = buf<unsigned long long>(h, h->scalars, 8);
    launch_fill_u64(reinterpret_cast<uint64_t *>(sc), 8, 0ull, st);
    void *tmp = h->arena.ensure(h->scan_tmp, scan_tmp_bytes(std::max<int64_t>(P, E) + 1));
    uint32_t *bmem = buf<uint32_t>(h, h->bmem, (size_t)std::max<int64_t>(E, 1));
    slot_t *bslot = buf<slot_t>(h, h->bslot, (size_t)std::max<int64_t>(E, 1));
    int64_t *pos_of = buf<int64_t>(h, h->pos_of, (size_t)std::max<int64_t>(E, 1));
    int64_t *bent = buf<int64_t>(h, h->bent, (size_t)std::max<int64_t>(E, 1));
    const bool radix = E > 0 && E < ((int64_t)1 << 32) &&
                       (h->bucket_build == 2 || (h->bucket_build == 0 && E >= kRadixMinEntries));
    if (radix) {
        // vertices in (priority, index) order, their entries in that order,
        // then a stable sort by colour: sorted buckets in one pass per digit
        uint32_t *k32a = buf<uint32_t>(h, h->rx_k32a, (size_t)m), *k32b = buf<uint32_t>(h, h->rx_k32b, (size_t)m);
        uint32_t *va = buf<uint32_t>(h, h->rx_va, (size_t)m), *vb = buf<uint32_t>(h, h->rx_vb, (size_t)m);
        void *rtmp = h->arena.ensure(h->rx_tmp, radix_tmp_bytes(std::max<int64_t>(m, E)));
        launch_prio_keys(prio, m, k32a, va, st);
        const int f1 = radix_sort_pairs<uint32_t>(k32a, va, k32b, vb, m, 0, 32, rtmp, st);
        uint32_t *perm = f1 ? vb : va;
        launch_prio_ties(f1 ? k32b : k32a, perm, prio, m, st);
        int32_t *tr = buf<int32_t>(h, h->rx_tr, (size_t)m);
        int64_t *at = buf<int64_t>(h, h->rx_at, (size_t)m + 1);
        launch_ranked_sizes(perm, m, b.loff, tr, st);
        exclusive_scan_i32_to_i64(tr, at, m, true, tmp, st);
        uint32_t *cka = buf<uint32_t>(h, h->rx_cka, (size_t)E), *ckb = buf<uint32_t>(h, h->rx_ckb, (size_t)E);
        uint32_t *cva = buf<uint32_t>(h, h->rx_cva, (size_t)E), *cvb = buf<uint32_t>(h, h->rx_cvb, (size_t)E);
        launch_emit_ranked(perm, m, b.loff, at, lists, cka, cva, E, st);
        int bits = 1;
        while (bits < 32 && ((int64_t)1 << bits) < P) ++bits;
        const int f2 = radix_sort_pairs<uint32_t>(cka, cva, ckb, cvb, E, 0, bits, rtmp, st);
        launch_bucket_from_sorted(b, f2 ? ckb : cka, f2 ? cvb : cva, E, P, bstart, bcnt, bmem, bslot, pos_of, bent,
                                  st);
        launch_bucket_pairs(bcnt, P, sc, st);
    } else {
        launch_fill_u32(bcnt, P, 0u, st);
        launch_bucket_count(lists, E, bcnt, st);
        launch_bucket_pairs(bcnt, P, sc, st);
        exclusive_scan_u32_to_i64(bcnt, bstart, P, true, tmp, st);
        launch_fill_u32(bcnt, P, 0u, st);
        launch_bucket_scatter(lists, m, b.loff, bstart, bcnt, bmem, bslot, st);
    }
    int32_t *binst = buf<int32_t>(h, h->binst, (size_t)P);
    launch_bucket_table(b, P, binst, st);
    b.binst = binst;
    // matrix shapes and their offsets (they depend on the bucket sizes only),
    // so that one round trip brings every total the host needs
    int64_t *tiles = buf<int64_t>(h, h->tiles, (size_t)P);
    int64_t *words = buf<int64_t>(h, h->words, (size_t)P);
    int64_t *tile_off = buf<int64_t>(h, h->tile_off, (size_t)P + 1);
    int64_t *rb_off = buf<int64_t>(h, h->rb_off, (size_t)P + 1);
    launch_bucket_shapes(bstart, P, tiles, words, st);
    exclusive_scan_i64(tiles, tile_off, P, true, tmp, st);
    exclusive_scan_i64(words, rb_off, P, true, tmp, st);
    unsigned long long hs[2];
    int64_t t2[2];
    PCHECK_HIP(hipMemcpyAsync(hs, sc, sizeof(hs), hipMemcpyDeviceToHost, st));
    PCHECK_HIP(hipMemcpyAsync(&t2[0], tile_off + P, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    PCHECK_HIP(hipMemcpyAsync(&t2[1], rb_off + P, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    if (d_hits)
        PCHECK_HIP(hipMemcpyAsync(h_hits, d_hits, sizeof(uint32_t) * (size_t)b.nb, hipMemcpyDeviceToHost, st));
    PCHECK_HIP(hipStreamSynchronize(st));
    BucketInfo bi;
    bi.pair_tests = (int64_t)hs[0];
    bi.max_size = (int64_t)hs[1];
    bi.row_tiles = t2[0];
    bi.words = t2[1];
    if (bi.max_size > (int64_t)1 << 17)
        throw Error(PICASSO_EINVAL, "a colour bucket holds " + std::to_string(bi.max_size) +
                                        " vertices (limit 131072): palette too small for this many vertices");
    if (!radix) {
        const bool large = bi.max_size > 2048;
        uint32_t *tmem = large ? buf<uint32_t>(h, h->tmp_mem, (size_t)E) : nullptr;
        slot_t *tslot = large ? buf<slot_t>(h, h->tmp_slot, (size_t)E) : nullptr;
        launch_bucket_sort(bstart, P, bmem, bslot, prio, pos_of, bent, b.loff, large, tmem, tslot, st);
    }
    return bi;
}

// Lists, priorities and buckets of one iteration.
BucketInfo build_lists_and_buckets(picasso_ctx *h, Batch &b, uint32_t ell, int64_t m, const int32_t *d_ids, int64_t E,
                                   int64_t P, int32_t T_max, const uint32_t *d_hits = nullptr,
                                   uint32_t *h_hits = nullptr)
{
    uint32_t *lists = buf<uint32_t>(h, h->lists, (size_t)std::max<int64_t>(E, 1));
    uint64_t *prio = buf<uint64_t>(h, h->prio, (size_t)std::max<int64_t>(m, 1));
    launch_sample_lists(b, ell, m, d_ids, T_max, lists, prio, h->stream);
    return buckets_from_lists(h, b, m, E, P, d_hits, h_hits);
}

// Upper bound on an iteration's conflict edges before the pair pass, from
// each instance's sampled relation density rho (K keyed vertex pairs).  A
// relation pair is a conflict edge when the two lists share a colour (Alg. 1
// construct_conflict_graph), and two uniform T-subsets of P colours meet with
// probability s = 1 - C(P-T, T) / C(P, T), so E|E_c| = C(m, 2) rho s.  The
// indicators of two pairs are independent even when the pairs share a
// vertex (a uniform T-subset meets every fixed T-subset with the same
// probability s), so |E_c| has variance C(m, 2) rho s (1 - s).  The bound
// takes rho four standard errors high, adds six standard deviations of
// |E_c|, and is never above the iteration's pair tests, which bound |E_c|
// exactly (each edge is a pair of the bucket of its smallest shared colour).
int64_t conflict_edge_bound(const std::vector<InstRec> &recs, const uint32_t *hits, int32_t K, int64_t pair_tests)
{
    double total = 0.0;
    for (size_t a = 0; a < recs.size(); ++a) {
        const InstRec &r = recs[a];
        if (r.m < 2) continue;
        const double m = (double)r.m, P = (double)r.P, T = (double)r.T;
        double share = 1.0;
        if (2.0 * T <= P)
            share = 1.0 - std::exp(2.0 * std::lgamma(P - T + 1.0) - std::lgamma(P - 2.0 * T + 1.0) -
                                   std::lgamma(P + 1.0));
        const double rho = (double)hits[a] / (double)K;
        const double rho_hi =
            std::min(1.0, rho + 4.0 * std::sqrt(std::max(rho * (1.0 - rho), 1.0 / K) / (double)K));
        const double mu = 0.5 * m * (m - 1.0) * rho_hi * share;
        total += mu + 6.0 * std::sqrt(mu * (1.0 - share)) + 64.0;
    }
    const double capped = std::min(total, (double)pair_tests);
    return (int64_t)std::ceil(capped);
}

// The CSR passes' arguments over the current buckets and matrices (the
// slot offsets as last scanned; no adjacency buffer, no skip flag).
CsrArgs csr_args(picasso_ctx *h, const Batch &b, int64_t P)
{
    CsrArgs ca{};
    ca.bstart = static_cast<const int64_t *>(h->bstart.p);
    ca.bmem = static_cast<const uint32_t *>(h->bmem.p);
    ca.bslot = static_cast<const slot_t *>(h->bslot.p);
    ca.P = P;
    ca.rb_off = static_cast<const int64_t *>(h->rb_off.p);
    ca.R = static_cast<const uint64_t *>(h->R.p);
    ca.D = static_cast<const uint64_t *>(h->D.p);
    ca.dflag = static_cast<const uint8_t *>(h->dflag.p);
    ca.loff = b.loff;
    ca.seg = static_cast<int32_t *>(h->seg.p);
    ca.seg_off = static_cast<const int64_t *>(h->seg_off.p);
    ca.seg_m = h->seg_m;
    ca.v_lo = 0;
    ca.v_hi = INT64_MAX;
    ca.adj_base = 0;
    return ca;
}

// Relation matrices, duplicate-pair matrices, CSR counts, scan and fill.
// rel_mask bit r: some instance of the batch uses relation r.  Returns
// |E_c|; the CSR is in h->rowptr / h->adj, each member's CSR position in
// h->seg_off (slot-major, stride h->seg_m).
int64_t build_conflict_graph(picasso_ctx *h, const Batch &b, int64_t m, int64_t E, int64_t P, int32_t T_max,
                             int32_t rel_mask, const BucketInfo &bi, double *ms_relate, double *ms_csr,
                             bool *used_mfma = nullptr, bool csr_required = true, int64_t edge_bound = -1,
                             bool want_edges = true)
{
    hipStream_t st = h->stream;
    Timer tm(h);
    uint64_t *R = buf<uint64_t>(h, h->R, (size_t)std::max<int64_t>(bi.words, 1));
    uint64_t *D = buf<uint64_t>(h, h->D, (size_t)std::max<int64_t>(bi.words, 1));
    RelateArgs ra{};
    ra.bstart = static_cast<const int64_t *>(h->bstart.p);
    ra.bmem = static_cast<const uint32_t *>(h->bmem.p);
    ra.P = P;
    ra.tile_off = static_cast<const int64_t *>(h->tile_off.p);
    ra.total_row_tiles = bi.row_tiles;
    ra.rb_off = static_cast<const int64_t *>(h->rb_off.p);
    ra.ids = static_cast<const int32_t *>(h->ids.p);
    ra.xz = static_cast<const uint64_t *>(h->xz.p);
    ra.W = h->W;
    ra.binst = b.binst;
    ra.inst = b.inst;
    ra.R = R;
    launch_relate_prep(ra, E, buf<uint64_t>(h, h->bx, (size_t)std::max<int64_t>(E, 1) * h->W),
                       buf<uint64_t>(h, h->bz, (size_t)std::max<int64_t>(E, 1) * h->W),
                       buf<int32_t>(h, h->tile_bucket, (size_t)std::max<int64_t>(bi.row_tiles, 1)), st);
    bool any_mfma = false;
    tm.mark();
    for (int32_t rel = 0; rel < 3; ++rel) {
        if (!(rel_mask >> rel & 1)) continue;
        // auto takes the popcount kernel, the faster one on every measured
        // workload; the MFMA kernel runs on request (or when the tuner picks it)
        const bool mfma = h->pair_path == PICASSO_PATH_MFMA;
        if (mfma && !mfma_supported(h->q, rel))
            throw Error(PICASSO_EINVAL, "the MFMA pair path does not support this q and relation");
        ra.relation = rel;
        ra.mfma_max_members = -1;
        if (mfma) {
            ra.mfma_max_members = mfma_member_cap(h->q, rel);
            if (h->mfma_cap >= 0 && h->mfma_cap < ra.mfma_max_members) ra.mfma_max_members = h->mfma_cap;
            // no larger than the largest bucket: the kernel's LDS is sized by
            // this bound, and a smaller one fits more workgroups per CU
            ra.mfma_max_members = std::min<int64_t>(ra.mfma_max_members, std::max<int64_t>(bi.max_size, 1));
        }
        any_mfma |= mfma;
        if (mfma) launch_relate_mfma(ra, h->q, st);
        if (!mfma || bi.max_size > ra.mfma_max_members) launch_relate(ra, st);
    }
    if (used_mfma) *used_mfma = any_mfma;
    tm.mark();
    if (!want_edges) {
        // the colouring reads the relation matrices only
        if (ms_relate) *ms_relate = tm.ms(0, 1);
        if (ms_csr) *ms_csr = 0.0;
        return -1;
    }
    // pairs sharing a smaller colour
    launch_fill_u64(D, bi.words, 0ull, st);
    uint8_t *dflag = buf<uint8_t>(h, h->dflag, (size_t)std::max<int64_t>(E, 1));
    launch_fill_u8(dflag, E, 0, st);
    int32_t *nslow = buf<int32_t>(h, h->nslow, 16);
    launch_fill_i32(nslow, 1, 0, st);
    DupArgs da{};
    da.bstart = ra.bstart;
    da.bmem = ra.bmem;
    da.bslot = static_cast<const slot_t *>(h->bslot.p);
    da.P = P;
    da.rb_off = ra.rb_off;
    da.lists = static_cast<const uint32_t *>(h->lists.p);
    da.loff = b.loff;
    da.bent = static_cast<const int64_t *>(h->bent.p);
    da.binst = b.binst;
    da.inst = b.inst;
    da.R = R;
    da.D = D;
    da.dflag = dflag;
    da.slow = buf<uint32_t>(h, h->slow, (size_t)P);
    da.n_slow = nslow;
    if (T_max > 1) {
        launch_dup(da, st);
        launch_dup_slow(da, st);  // its bucket count is read on the device
    }
    // edge counts per (vertex, slot), row lengths, row pointers from their
    // scan, and each segment's CSR position
    const size_t nseg = (size_t)std::max<int64_t>((int64_t)T_max * m, 1);
    buf<int32_t>(h, h->seg, nseg);
    buf<int64_t>(h, h->seg_off, nseg);
    h->seg_m = m;
    int64_t *rowptr = buf<int64_t>(h, h->rowptr, (size_t)m + 1);
    CsrArgs ca = csr_args(h, b, P);
    launch_count(ca, st);
    int32_t *deg = buf<int32_t>(h, h->deg, (size_t)std::max<int64_t>(m, 1));
    launch_row_lengths(ca.seg, m, b.loff, deg, st);
    void *tmp = h->arena.ensure(h->scan_tmp, scan_tmp_bytes(std::max<int64_t>(P, E) + 1));
    exclusive_scan_i32_to_i64(deg, rowptr, m, true, tmp, st);
    launch_seg_offsets(ca.seg, m, b.loff, rowptr, static_cast<int64_t *>(h->seg_off.p), st);
    if (edge_bound >= 0 && !csr_required &&
        (h->mem_budget <= 0 || 2 * edge_bound * (int64_t)sizeof(int32_t) <= h->mem_budget)) {
        // CSR sized by the predicted bound: the fill is queued without waiting
        // for the exact size; a guard on the device skips it if the size
        // exceeds the buffer (the caller refills once it knows the size)
        const int64_t cap = 2 * edge_bound;
        ca.adj = buf<int32_t>(h, h->adj, (size_t)std::max<int64_t>(cap, 1));
        int32_t *flag = buf<int32_t>(h, h->csr_flag, 1);
        launch_csr_guard(rowptr + m, cap, flag, st);
        ca.skip = flag;
        tm.mark();
        launch_fill(ca, bi.max_size, st);
        tm.mark();
        if (ms_relate) *ms_relate = tm.ms(0, 1);
        if (ms_csr) *ms_csr = tm.ms(2, 3);
        return -1;
    }
    const int64_t total = read_scalar(h, rowptr + m);
    if (total % 2) throw Error(PICASSO_EINTERNAL, "odd CSR size");
    const int64_t bytes = total * (int64_t)sizeof(int32_t);
    if (h->mem_budget > 0 && bytes > h->mem_budget) {
        if (csr_required)
            throw Error(PICASSO_ENOMEM, "conflict graph needs " + std::to_string(bytes) + " bytes, budget " +
                                            std::to_string(h->mem_budget));
        // the colouring reads the bucket relation matrices, not the CSR: the
        // edges are counted and the adjacency is not written
        if (ms_relate) *ms_relate = tm.ms(0, 1);
        if (ms_csr) *ms_csr = 0.0;
        return total / 2;
    }
    ca.adj = buf<int32_t>(h, h->adj, (size_t)std::max<int64_t>(total, 1));
    tm.mark();
    launch_fill(ca, bi.max_size, st);
    tm.mark();
    if (ms_relate) *ms_relate = tm.ms(0, 1);
    if (ms_csr) *ms_csr = tm.ms(2, 3);
    return total / 2;
}

// The CSR of the last build_conflict_graph written to the host in chunks of
// whole rows, each at most the memory budget: chunk [v0, v1) is filled on the
// device from the bucket matrices (rows of other vertices skipped) and copied
// to out_adj[rowptr[v0] .. rowptr[v1]).  rowptr: host copy of the row
// pointers.  ENOMEM if one row alone exceeds the budget.
void fill_csr_chunks(picasso_ctx *h, const Batch &b, int64_t m, int64_t P, const BucketInfo &bi, const int64_t *rowptr,
                     int32_t *out_adj)
{
    const int64_t cap = h->mem_budget / (int64_t)sizeof(int32_t);
    const int64_t total = rowptr[m];
    int32_t *chunk = buf<int32_t>(h, h->adj, (size_t)std::max<int64_t>(std::min(cap, total), 1));
    CsrArgs ca = csr_args(h, b, P);
    ca.adj = chunk;
    for (int64_t v0 = 0; v0 < m;) {
        // the longest run of rows from v0 within the budget
        const int64_t *end = std::upper_bound(rowptr + v0, rowptr + m + 1, rowptr[v0] + cap);
        const int64_t v1 = (int64_t)(end - rowptr) - 1;
        if (v1 <= v0)
            throw Error(PICASSO_ENOMEM, "row " + std::to_string(v0) + " of the conflict graph needs " +
                                            std::to_string((rowptr[v0 + 1] - rowptr[v0]) * 4) + " bytes, budget " +
                                            std::to_string(h->mem_budget));
        ca.v_lo = v0;
        ca.v_hi = v1;
        ca.adj_base = rowptr[v0];
        launch_fill(ca, bi.max_size, h->stream);
        download(h, out_adj + rowptr[v0], chunk, (size_t)(rowptr[v1] - rowptr[v0]) * sizeof(int32_t));
        v0 = v1;
    }
}

// Colouring rounds: `count` rounds starting from worklist `cur`, either
// launched one by one or replayed from a graph captured once per
// iteration (the rounds' arguments do not change within an iteration).
struct RoundGraph {
    hipGraphExec_t exec[2] = {nullptr, nullptr};  // starting from list 0 / list 1, captured on first use
    int32_t rounds = 0;
    ~RoundGraph()
    {
        for (auto &e : exec)
            if (e) (void)hipGraphExecDestroy(e);
    }
};

// One batch of rounds from list `start`: begin, the rounds, end.
void launch_jp_batch(picasso_ctx *h, const JpArgs &j, int32_t rounds, int start)
{
    launch_jp_batch_begin(j, rounds, h->stream);
    int cur = start;
    for (int32_t r = 0; r < rounds; ++r) {
        launch_jp_round(j, cur, r, h->stream);
        cur ^= 1;
    }
    launch_jp_batch_end(j, rounds, h->stream);
}

void capture_rounds(picasso_ctx *h, const JpArgs &j, RoundGraph &g, int32_t rounds, int start)
{
    hipGraph_t graph = nullptr;
    PCHECK_HIP(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
    try {
        launch_jp_batch(h, j, rounds, start);
    } catch (...) {
        (void)hipStreamEndCapture(h->stream, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        throw;
    }
    PCHECK_HIP(hipStreamEndCapture(h->stream, &graph));
    const hipError_t e = hipGraphInstantiate(&g.exec[start], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    PCHECK_HIP(e);
    g.rounds = rounds;
}

// List colouring until every vertex is decided.  Result in h->col.
int32_t color_buckets(picasso_ctx *h, const Batch &b, int64_t m, int64_t E, int64_t P, int32_t T_max,
                      const BucketInfo &bi)
{
    hipStream_t st = h->stream;
    JpArgs j{};
    j.P = P;
    j.bstart = static_cast<const int64_t *>(h->bstart.p);
    j.bmem = static_cast<const uint32_t *>(h->bmem.p);
    j.bslot = static_cast<const slot_t *>(h->bslot.p);
    j.rb_off = static_cast<const int64_t *>(h->rb_off.p);
    j.R = static_cast<const uint64_t *>(h->R.p);
    j.lists = static_cast<const uint32_t *>(h->lists.p);
    j.loff = b.loff;
    j.pos_of = static_cast<const int64_t *>(h->pos_of.p);
    j.inst = b.inst;
    j.binst = b.binst;
    j.nw_max = std::max<int64_t>((bi.max_size + 63) / 64, 1);
    j.fw = (T_max + 63) / 64;
    j.col = buf<int32_t>(h, h->col, (size_t)std::max<int64_t>(m, 1));
    j.packed = T_max <= 32;
    j.blk = buf<uint64_t>(h, h->blk, (size_t)m * j.fw);
    if (!j.packed) {
        j.fre = buf<uint64_t>(h, h->fre, (size_t)m * j.fw);
        j.nblk = buf<int32_t>(h, h->nblk, (size_t)std::max<int64_t>(m, 1));
    }
    j.st = buf<uint8_t>(h, h->st, (size_t)std::max<int64_t>(E, 1));
    j.rdy = buf<uint8_t>(h, h->rdy, (size_t)std::max<int64_t>(E, 1));
    j.wake_at = buf<unsigned long long>(h, h->wake_at, (size_t)P);
    j.wl_cap = (P + kJpSeg - 1) / kJpSeg;
    const int64_t wl_len = kJpSeg * j.wl_cap;
    int32_t *wl = buf<int32_t>(h, h->wl, (size_t)(2 * wl_len + (int64_t)kJpSlots * kJpRow));
    j.wl[0] = wl;
    j.wl[1] = wl + wl_len;
    j.wl_cnt = wl + 2 * wl_len;
    unsigned long long *prog = buf<unsigned long long>(h, h->jp_prog, (size_t)kJpSeg * kJpProgStride + 2);
    j.progress = prog;
    j.totals = prog + (size_t)kJpSeg * kJpProgStride;
    j.m = m;
    launch_fill_i32(j.col, m, COL_UNDECIDED, st);
    launch_fill_u64(j.blk, m * j.fw, 0ull, st);
    if (!j.packed) {
        launch_fill_u64(j.fre, m * j.fw, 0ull, st);
        launch_fill_i32(j.nblk, m, 0, st);
    }
    launch_fill_u8(j.st, E, 0, st);
    launch_fill_u8(j.rdy, E, 0, st);
    launch_fill_u64(reinterpret_cast<uint64_t *>(j.progress), (int64_t)kJpSeg * kJpProgStride + 2, 0ull, st);
    launch_jp_all(j, st);
    RoundGraph graph;
    const int32_t max_batch = std::max<int32_t>(h->jp_batch, 1);
    int32_t rounds = 0;
    // Rounds with nothing to do exit at once (a few us), so a whole batch
    // first costs less than host checks between smaller ones.  The first
    // batch is launched round by round: most iterations end within it, and
    // capturing the graph, done only for a second batch, costs more than
    // the launches it saves.
    int cur = 0, batch = max_batch;
    unsigned long long at_restart = 0;
    bool fresh = true;  // the lists hold every bucket
    while (true) {
        if (h->use_graph && batch == max_batch && max_batch > 1 && rounds > 0) {
            if (!graph.exec[cur]) capture_rounds(h, j, graph, batch, cur);
            PCHECK_HIP(hipGraphLaunch(graph.exec[cur], st));
            if (batch & 1) cur ^= 1;
        } else {
            launch_jp_batch(h, j, batch, cur);
            if (batch & 1) cur ^= 1;
        }
        rounds += batch;
        unsigned long long tot[2] = {0, 0};
        PCHECK_HIP(hipMemcpyAsync(tot, j.totals, sizeof(tot), hipMemcpyDeviceToHost, st));
        PCHECK_HIP(hipStreamSynchronize(st));
        const unsigned long long done = tot[0];
        const unsigned long long pending = tot[1];
        if ((int64_t)done >= m) break;
        if (pending == 0) {
            // Nothing left on the worklist but vertices remain: start again
            // from every bucket.  Rounds that start from every bucket decide
            // at least the first undecided vertex of the order.
            if (fresh && done == at_restart) throw Error(PICASSO_EINTERNAL, "list colouring made no progress");
            at_restart = done;
            launch_jp_all(j, st);
            cur = 0;
            fresh = true;
        } else {
            fresh = false;
        }
        batch = std::min<int32_t>(batch * 2, max_batch);
    }
    return rounds;
}

// Dynamic-order colouring (the round form of Alg. 2) until every vertex is
// coloured or has lost its whole list.  Result in h->col; returns rounds.
int32_t color_buckets_dynamic(picasso_ctx *h, const Batch &b, uint32_t ell, int64_t m, int64_t E, int64_t P,
                              int32_t T_max, const BucketInfo &bi)
{
    hipStream_t st = h->stream;
    DynArgs a{};
    a.b = b;
    a.m = m;
    a.P = P;
    a.ids = static_cast<const int32_t *>(h->ids.p);
    a.pos_of = static_cast<const int64_t *>(h->pos_of.p);
    a.bstart = static_cast<const int64_t *>(h->bstart.p);
    a.bmem = static_cast<const uint32_t *>(h->bmem.p);
    a.bslot = static_cast<const slot_t *>(h->bslot.p);
    a.rb_off = static_cast<const int64_t *>(h->rb_off.p);
    a.R = static_cast<const uint64_t *>(h->R.p);
    a.nw_max = std::max<int64_t>((bi.max_size + 63) / 64, 1);
    a.fw = (T_max + 63) / 64;
    a.alive = buf<uint64_t>(h, h->blk, (size_t)m * a.fw);
    a.size = buf<int32_t>(h, h->nblk, (size_t)std::max<int64_t>(m, 1));
    a.col = buf<int32_t>(h, h->col, (size_t)std::max<int64_t>(m, 1));
    a.rkey = buf<uint64_t>(h, h->rkey, (size_t)std::max<int64_t>(m, 1));
    a.st = buf<uint8_t>(h, h->st, (size_t)std::max<int64_t>(E, 1));
    a.hist_w = T_max + 1;
    a.hist = buf<unsigned long long>(h, h->dyn_hist, (size_t)b.nb * a.hist_w);
    a.sstar = buf<int32_t>(h, h->dyn_sstar, (size_t)b.nb);
    a.cut = buf<uint64_t>(h, h->dyn_cut, (size_t)b.nb);
    a.active = buf<unsigned long long>(h, h->scalars, 8) + 6;
    a.divisor = h->dyn_divisor;
    a.ell = ell;
    launch_fill_u8(a.st, E, 0, st);
    launch_fill_u64(reinterpret_cast<uint64_t *>(a.hist), (int64_t)b.nb * a.hist_w, 0ull, st);
    launch_dyn_init(a, st);
    // every round with an active vertex colours at least the first requester
    // of each requested colour, so m rounds always suffice
    const int64_t max_rounds = m + 64;
    int32_t round = 0, batch = 4;
    while (true) {
        for (int r = 0; r < batch; ++r) launch_dyn_round(a, round++, st);
        unsigned long long active = 0;
        PCHECK_HIP(hipMemcpyAsync(&active, a.active, sizeof(active), hipMemcpyDeviceToHost, st));
        PCHECK_HIP(hipStreamSynchronize(st));
        if (active == 0) break;
        if (round > max_rounds) throw Error(PICASSO_EINTERNAL, "dynamic colouring made no progress");
        batch = std::min<int32_t>(batch * 2, std::max<int32_t>(h->jp_batch, 1));
    }
    return round;
}

void init_ids(picasso_ctx *h, int64_t m);

// Features of the m vertices at d_ids (one instance with q qubits): exact
// integer counts from the device, the five values formed on the host in
// double.
void device_features(picasso_ctx *h, uint64_t seed, uint32_t ell, int64_t m, const int32_t *d_ids, int32_t q,
                     int32_t rel, double out[5])
{
    unsigned long long *sc = buf<unsigned long long>(h, h->scalars, 8);
    launch_fill_u64(reinterpret_cast<uint64_t *>(sc + 4), 2, 0ull, h->stream);
    launch_features(m, d_ids, static_cast<const uint64_t *>(h->x.p), static_cast<const uint64_t *>(h->z.p), h->W,
                    seed, ell, rel, kFeaturePairs, sc + 4, sc + 5, h->stream);
    unsigned long long hv[2];
    PCHECK_HIP(hipMemcpyAsync(hv, sc + 4, sizeof(hv), hipMemcpyDeviceToHost, h->stream));
    PCHECK_HIP(hipStreamSynchronize(h->stream));
    out[0] = m > 0 ? std::log((double)m) : 0.0;
    out[1] = (double)q;
    out[2] = m > 0 ? (double)hv[0] / (double)m : 0.0;
    out[3] = m >= 2 ? (double)hv[1] / (double)kFeaturePairs : 0.0;
    out[4] = (double)ell;
}

// The predictor's (f, alpha) for one feature row (five features and beta),
// computed on the device.
void mlp_params_for(picasso_mlp_ctx *mc, hipStream_t st, const double feat[kMlpIn], float fa_out[2])
{
    float raw[kMlpIn];
    for (int i = 0; i < kMlpIn; ++i) raw[i] = (float)feat[i];
    float *d_raw = mbuf<float>(mc, mc->raw, 8);
    float *d_out = mbuf<float>(mc, mc->out, 8);
    float *d_fa = mbuf<float>(mc, mc->fa, 8);
    PCHECK_HIP(hipMemcpyAsync(d_raw, raw, sizeof(raw), hipMemcpyHostToDevice, st));
    launch_mlp_rows(static_cast<const float *>(mc->params.p), d_raw, 1, d_out, nullptr, nullptr, nullptr, st);
    launch_squash(d_out, 1, d_fa, st);
    PCHECK_HIP(hipMemcpyAsync(fa_out, d_fa, 2 * sizeof(float), hipMemcpyDeviceToHost, st));
    PCHECK_HIP(hipStreamSynchronize(st));
}

// Per-instance run arguments of one colouring call.
struct RunArgs {
    const uint64_t *seeds;
    const double *fracs, *alphas;
    const int32_t *rels;
    picasso_mlp_ctx *mlp = nullptr;  // learned parameters (single-instance calls)
    float *sched = nullptr;          // the learned (f, alpha) of each iteration
    int32_t max_sched = 0;
    double beta = 0.5;               // the network's trade-off input
    // explicit schedule (single-instance calls): iteration l uses entry
    // min(l, n_steps) - 1; fracs/alphas then point at the last entry
    const double *step_f = nullptr, *step_a = nullptr;
    int32_t n_steps = 0;
};

// Adds one iteration's record (one instance's share, or the whole batch's)
// to the call's statistics; iteration `idx` counts from 0.
void add_iter(picasso_stats &S, std::vector<int64_t> &iter_edges, int64_t idx, const picasso_iter_stats &it)
{
    if ((int64_t)iter_edges.size() <= idx) iter_edges.resize((size_t)idx + 1, 0);
    iter_edges[(size_t)idx] += it.edges;
    if (idx < PICASSO_MAX_ITER_STATS) {
        picasso_iter_stats &d = S.iters[idx];
        d.m += it.m;
        d.P += it.P;
        d.T = std::max(d.T, it.T);
        d.pair_tests += it.pair_tests;
        d.edges += it.edges;
        d.edges_bound += it.edges_bound;
        d.colored += it.colored;
        d.offset = it.offset;
        d.pair_path = std::max(d.pair_path, it.pair_path);
        d.jp_rounds += it.jp_rounds;
        d.ms_graph += it.ms_graph;
        d.ms_buckets += it.ms_buckets;
        d.ms_count += it.ms_count;
        d.ms_fill += it.ms_fill;
        d.ms_color += it.ms_color;
        d.ms_compact += it.ms_compact;
    }
    S.n_iters = std::max<int32_t>(S.n_iters, (int32_t)(idx + 1));
    S.palette_total += it.P;
    S.pair_tests += it.pair_tests;
    S.edges += it.edges;
}

// Whether every iteration of an instance with m vertices left fits the tail
// kernel's LDS; fills the instance's (P, T) table for 0..m vertices.
bool tail_table(int64_t m, double frac, double alpha, int32_t fixed_T, std::vector<int32_t> &table)
{
    const size_t at = table.size();
    table.resize(at + 2 * ((size_t)kTailMax + 1), 0);
    for (int64_t k = 1; k <= m; ++k) {
        int64_t P;
        int32_t T;
        params(k, frac, alpha, fixed_T, P, T);
        if (P > kTailMax || (int64_t)T * k > kTailListCap) {
            table.resize(at);
            return false;
        }
        table[at + 2 * k] = (int32_t)P;
        table[at + 2 * k + 1] = T;
    }
    return true;
}

// Tail launches of one colouring call.  Each launch finishes the instances
// that entered the tail in one iteration; it runs on the handle's tail stream
// beside the main path, from its own copy of the instances' vertex ids, and
// writes into its own slices of buffers sized for every instance (nothing is
// reused within the call).  Its records are read back once the call ends.
struct TailPlan {
    TailRec *recs = nullptr;
    int32_t *table = nullptr;
    TailOut *outs = nullptr;
    TailIter *iters = nullptr;
    int32_t *ids = nullptr;
    int64_t n_recs = 0, n_table = 0, n_ids = 0;
    struct Launch {
        uint32_t ell;
        int64_t rec0;
        std::vector<int32_t> tinst;
    };
    std::vector<Launch> launches;
    std::vector<std::vector<TailRec>> h_recs;     // host copies kept until the call ends
    std::vector<std::vector<int32_t>> h_tables;
    std::vector<std::vector<int64_t>> h_ranges;
};

void tail_plan_init(picasso_ctx *h, TailPlan &tp)
{
    const size_t nb = (size_t)std::max<int32_t>(h->nb, 1);
    tp.recs = buf<TailRec>(h, h->tail_recs, nb);
    tp.table = buf<int32_t>(h, h->tail_table, nb * 2 * ((size_t)kTailMax + 1));
    tp.outs = buf<TailOut>(h, h->tail_outs, nb);
    tp.iters = buf<TailIter>(h, h->tail_iters, nb * kTailMax);
    tp.ids = buf<int32_t>(h, h->tail_ids, nb * kTailMax);
    if (!h->tail_stream) {
        PCHECK_HIP(hipStreamCreateWithFlags(&h->tail_stream, hipStreamNonBlocking));
        PCHECK_HIP(hipEventCreateWithFlags(&h->tail_ready, hipEventDisableTiming));
        PCHECK_HIP(hipEventCreateWithFlags(&h->tail_done, hipEventDisableTiming));
    }
}

// Hands the active instances with at most kTailMax vertices left (and every
// iteration within the tail kernel's limits) to the tail kernel, which
// finishes them; the other instances' vertices (contiguous runs of
// h->next_ids) are gathered to the front of h->ids when some left.  Returns
// the vertices left for the next iteration; the finished instances' mi
// become 0 (their colours and statistics are collected by tail_plan_finish).
int64_t run_tails(picasso_ctx *h, const RunArgs &ra, const std::vector<int32_t> &act, std::vector<int64_t> &mi,
                  const std::vector<int64_t> &off, uint32_t ell, int32_t *d_out, TailPlan &tp, bool &gathered)
{
    hipStream_t st = h->stream;
    std::vector<TailRec> trs;
    std::vector<int32_t> tinst, table;
    std::vector<int64_t> ranges, tranges;
    int64_t src = 0, kept = 0, tcopy = 0;
    for (const int32_t i : act) {
        const int64_t mn = mi[i];
        if (mn > 0 && mn <= kTailMax && tail_table(mn, ra.fracs[i], ra.alphas[i], h->fixed_T, table)) {
            TailRec tr{};
            tr.src = tcopy;  // in this launch's copy of the ids
            tr.m = mn;
            tr.sbase = h->inst_base[i];
            tr.cbase = off[i];
            tr.seed = ra.seeds[i];
            tr.ell = (int32_t)ell + 1;
            tr.rel = ra.rels[i];
            tr.table = (int32_t)(table.size() - 2 * ((size_t)kTailMax + 1));
            tr.iter0 = (int32_t)(trs.size() * kTailMax);
            trs.push_back(tr);
            tinst.push_back(i);
            tranges.push_back(src);
            tranges.push_back(tcopy);
            tcopy += mn;
        } else if (mn > 0) {
            ranges.push_back(src);
            ranges.push_back(kept);
            kept += mn;
        }
        src += mn;
    }
    gathered = false;
    if (trs.empty()) return kept;
    const int32_t nt = (int32_t)trs.size();
    if (tp.n_recs + nt > std::max<int32_t>(h->nb, 1) || tp.n_ids + tcopy > (int64_t)std::max<int32_t>(h->nb, 1) * kTailMax ||
        tp.n_table + (int64_t)table.size() > (int64_t)std::max<int32_t>(h->nb, 1) * 2 * (kTailMax + 1))
        throw Error(PICASSO_EINTERNAL, "tail buffers exceeded");
    TailRec *d_recs = tp.recs + tp.n_recs;
    int32_t *d_table = tp.table + tp.n_table;
    int32_t *d_ids = tp.ids + tp.n_ids;
    const int32_t *next = static_cast<const int32_t *>(h->next_ids.p);
    // the tail instances' vertex ids, copied (the main path rewrites next_ids)
    int64_t *d_tr = buf<int64_t>(h, h->tail_ranges, ranges.size() + tranges.size());
    upload(h, d_tr, tranges.data(), tranges.size() * sizeof(int64_t));
    launch_gather_ranges(next, d_ids, d_tr, (int32_t)(tranges.size() / 2), tcopy, st);
    upload(h, d_recs, trs.data(), trs.size() * sizeof(TailRec));
    upload(h, d_table, table.data(), table.size() * sizeof(int32_t));
    if (kept > 0) {
        int64_t *d_ranges = d_tr + tranges.size();
        upload(h, d_ranges, ranges.data(), ranges.size() * sizeof(int64_t));
        int32_t *ids = buf<int32_t>(h, h->ids, (size_t)kept);
        launch_gather_ranges(next, ids, d_ranges, (int32_t)(ranges.size() / 2), kept, st);
        gathered = true;
    }
    // the copies and uploads are complete before the tail stream starts
    PCHECK_HIP(hipEventRecord(h->tail_ready, st));
    PCHECK_HIP(hipStreamWaitEvent(h->tail_stream, h->tail_ready, 0));
    launch_tail(d_recs, nt, d_ids, static_cast<const uint64_t *>(h->xz.p), h->W, d_table, d_out, tp.outs + tp.n_recs,
                tp.iters + tp.n_recs * kTailMax, h->tail_stream);
    // d_tr is reused by the next launch's uploads: the gathers that read it
    // are on the main stream, ordered before those uploads
    tp.launches.push_back({ell, tp.n_recs, tinst});
    tp.n_recs += nt;
    tp.n_table += (int64_t)table.size();
    tp.n_ids += tcopy;
    tp.h_recs.push_back(std::move(trs));
    tp.h_tables.push_back(std::move(table));
    tp.h_ranges.push_back(std::move(tranges));
    tp.h_ranges.push_back(std::move(ranges));
    for (const int32_t i : tinst) mi[i] = 0;
    return kept;
}

// Waits for the tail launches (the main stream waits on the tail stream) and
// adds their colour counts and iteration records.
void tail_plan_finish(picasso_ctx *h, TailPlan &tp, std::vector<int64_t> &off, int64_t *n_colors, picasso_stats &S,
                      std::vector<int64_t> &iter_edges)
{
    if (tp.launches.empty()) return;
    PCHECK_HIP(hipEventRecord(h->tail_done, h->tail_stream));
    PCHECK_HIP(hipStreamWaitEvent(h->stream, h->tail_done, 0));
    std::vector<TailOut> outs((size_t)tp.n_recs);
    std::vector<TailIter> its((size_t)tp.n_recs * kTailMax);
    download(h, outs.data(), tp.outs, outs.size() * sizeof(TailOut));
    download(h, its.data(), tp.iters, its.size() * sizeof(TailIter));
    for (const TailPlan::Launch &L : tp.launches) {
        for (size_t b = 0; b < L.tinst.size(); ++b) {
            const int32_t i = L.tinst[b];
            const int64_t r = L.rec0 + (int64_t)b;
            picasso_instance_stats &is = h->istats[i];
            n_colors[i] += outs[r].n_colors;
            for (int32_t j = 0; j < outs[r].n_iters; ++j) {
                const TailIter &ti = its[(size_t)r * kTailMax + j];
                picasso_iter_stats it{};
                it.m = ti.m;
                it.P = ti.P;
                it.T = ti.T;
                it.pair_tests = ti.pair_tests;
                it.edges = ti.edges;
                it.edges_bound = ti.edges;  // counted exactly, no CSR to size
                it.colored = ti.colored;
                it.offset = h->nb == 1 ? ti.offset : 0;
                it.pair_path = 0;
                add_iter(S, iter_edges, (int64_t)L.ell + j, it);
                off[i] += ti.P;
                is.n_iters++;
                is.palette_total += ti.P;
                is.edges += ti.edges;
                is.max_edges = std::max<int64_t>(is.max_edges, ti.edges);
            }
        }
    }
}

// Colours every instance of the handle (Alg. 1 loop, all instances side by
// side: iteration l advances every instance that still has uncoloured
// vertices).  Colours land in d_out at each string's packed index;
// n_colors[i] receives instance i's colour count.  Returns their sum.
int64_t color_all(picasso_ctx *h, const RunArgs &ra, int32_t *d_out, int64_t *n_colors)
{
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = h->stream;
    picasso_stats &S = h->stats;
    std::memset(&S, 0, sizeof(S));
    S.n = h->n;
    h->istats.assign((size_t)h->nb, picasso_instance_stats{});
    h->arena.peak = h->arena.live;
    launch_fill_i32(d_out, h->n, -1, st);
    init_ids(h, h->n);
    std::vector<int64_t> mi(h->inst_n), off((size_t)h->nb, 0);
    for (int32_t i = 0; i < h->nb; ++i) {
        n_colors[i] = 0;
        h->istats[i].n = h->inst_n[i];
    }
    std::vector<int32_t> act;
    std::vector<int64_t> hv, iter_edges;
    std::vector<uint32_t> h_hits;
    TailPlan tp;
    const bool tails = !ra.mlp && h->use_tail && h->colourer == PICASSO_COLOURER_STATIC;
    if (tails) tail_plan_init(h, tp);
    int64_t m = h->n;
    uint32_t ell = 1;
    while (m > 0) {
        // the active instances' table
        h->h_inst.clear();
        act.clear();
        int64_t vs = 0, E = 0, Ptot = 0;
        int32_t T_max = 0, rel_mask = 0;
        for (int32_t i = 0; i < h->nb; ++i) {
            if (mi[i] == 0) continue;
            double frac = ra.fracs[i], alpha = ra.alphas[i];
            if (ra.n_steps > 0) {
                const int32_t k = std::min<int32_t>((int32_t)ell, ra.n_steps) - 1;
                frac = ra.step_f[k];
                alpha = ra.step_a[k];
            } else if (ra.mlp) {
                double feat[kMlpIn];
                device_features(h, ra.seeds[i], ell, mi[i], static_cast<const int32_t *>(h->ids.p) + vs,
                                h->inst_q[i], ra.rels[i], feat);
                feat[5] = ra.beta;
                float fa[2];
                mlp_params_for(ra.mlp, h->stream, feat, fa);
                // fallback: an output outside the parameter ranges (only
                // corrupt weights give one) keeps the fixed parameters
                if (std::isfinite(fa[0]) && std::isfinite(fa[1]) && fa[0] > 0.f && fa[0] <= 1.f && fa[1] > 0.f) {
                    frac = (double)fa[0];
                    alpha = (double)fa[1];
                }
                if (ra.sched && (int32_t)ell <= ra.max_sched) {
                    ra.sched[2 * (ell - 1)] = fa[0];
                    ra.sched[2 * (ell - 1) + 1] = fa[1];
                }
            }
            int64_t P;
            int32_t T;
            params(mi[i], frac, alpha, h->fixed_T, P, T);
            if (T > PICASSO_MAX_T)
                throw Error(PICASSO_EINVAL, "list size " + std::to_string(T) + " exceeds PICASSO_MAX_T");
            InstRec r{};
            r.vstart = vs;
            r.m = mi[i];
            r.loff = E;
            r.pal = Ptot;
            r.P = P;
            r.sbase = h->inst_base[i];
            r.cbase = off[i];
            r.seed = ra.seeds[i];
            r.T = T;
            r.rel = ra.rels[i];
            h->h_inst.push_back(r);
            act.push_back(i);
            vs += mi[i];
            E += mi[i] * T;
            Ptot += P;
            T_max = std::max(T_max, T);
            rel_mask |= 1 << ra.rels[i];
        }
        if (Ptot > INT32_MAX) throw Error(PICASSO_EINVAL, "palette too large");
        picasso_iter_stats it{};
        it.m = m;
        it.P = Ptot;
        it.T = T_max;
        it.offset = h->nb == 1 ? off[0] : 0;
        Timer tm(h);
        tm.mark();
        Batch b = upload_batch(h, m);
        const int32_t *d_ids = static_cast<const int32_t *>(h->ids.p);
        // sampled relation density per instance: the conflict-graph size
        // bound that sizes the CSR before the pair pass
        uint32_t *d_hits = buf<uint32_t>(h, h->hits, (size_t)b.nb);
        launch_fill_u32(d_hits, b.nb, 0u, st);
        launch_density(b, d_ids, static_cast<const uint64_t *>(h->x.p), static_cast<const uint64_t *>(h->z.p), h->W,
                       ell, kSizingPairs, d_hits, st);
        h_hits.resize((size_t)b.nb);
        const BucketInfo bi = build_lists_and_buckets(h, b, ell, m, d_ids, E, Ptot, T_max, d_hits, h_hits.data());
        it.pair_tests = bi.pair_tests;
        it.edges_bound = conflict_edge_bound(h->h_inst, h_hits.data(), kSizingPairs, bi.pair_tests);
        tm.mark();
        bool used_mfma = false;
        const int64_t presize = h->csr_sizing == 0 ? -1 : h->csr_sizing == 2 ? 0 : it.edges_bound;
        it.edges = build_conflict_graph(h, b, m, E, Ptot, T_max, rel_mask, bi, &it.ms_count, &it.ms_fill,
                                        &used_mfma, false, presize, h->edges_on != 0);
        const bool csr_deferred = h->edges_on && it.edges < 0;
        if (!h->edges_on) it.edges_bound = -1;
        it.pair_path = used_mfma ? PICASSO_PATH_MFMA : PICASSO_PATH_VALU;
        tm.mark();
        it.jp_rounds = h->colourer == PICASSO_COLOURER_DYNAMIC
                           ? color_buckets_dynamic(h, b, ell, m, E, Ptot, T_max, bi)
                           : color_buckets(h, b, m, E, Ptot, T_max, bi);
        tm.mark();
        // output colours, used-colour counts, next vertex set
        const int32_t na = b.nb;
        uint32_t *used = buf<uint32_t>(h, h->used, (size_t)(Ptot + 31) / 32);
        launch_fill_u32(used, (Ptot + 31) / 32, 0u, st);
        int64_t *iout = buf<int64_t>(h, h->inst_out, (size_t)3 * na);  // used, m_next, edges
        launch_fill_u64(reinterpret_cast<uint64_t *>(iout), 3 * na, 0ull, st);
        int32_t *flags = buf<int32_t>(h, h->flags, (size_t)m);
        launch_finish_iteration(b, m, static_cast<const int32_t *>(h->col.p), d_ids, d_out, used,
                                reinterpret_cast<unsigned long long *>(iout), flags, st);
        int64_t *pos = buf<int64_t>(h, h->pos, (size_t)m + 1);
        void *tmp = h->arena.ensure(h->scan_tmp, scan_tmp_bytes(std::max<int64_t>(Ptot, m)));
        exclusive_scan_i32_to_i64(flags, pos, m, true, tmp, st);
        int32_t *next = buf<int32_t>(h, h->next_ids, (size_t)m);
        launch_compact_ids(m, d_ids, flags, pos, next, st);
        launch_instance_totals(b, pos, static_cast<const int64_t *>(h->rowptr.p), iout + na,
                               h->edges_on ? iout + 2 * na : nullptr, st);
        tm.mark();
        hv.resize((size_t)3 * na);
        download(h, hv.data(), iout, hv.size() * sizeof(int64_t));
        if (csr_deferred) {
            it.edges = 0;
            for (int32_t a = 0; a < na; ++a) it.edges += hv[2 * na + a];
            if (it.edges > presize) {
                // above the predicted bound (the guard skipped the fill):
                // the CSR again at its exact size
                CsrArgs ca = csr_args(h, b, Ptot);
                ca.adj = buf<int32_t>(h, h->adj, (size_t)std::max<int64_t>(2 * it.edges, 1));
                launch_fill(ca, bi.max_size, st);
                PCHECK_HIP(hipStreamSynchronize(st));
                ++S.csr_refills;
            }
        }
        int64_t m_next = 0;
        for (int32_t a = 0; a < na; ++a) {
            const int32_t i = act[a];
            const InstRec &r = h->h_inst[a];
            picasso_instance_stats &is = h->istats[i];
            n_colors[i] += hv[a];
            mi[i] = hv[na + a];
            m_next += mi[i];
            off[i] += r.P;
            is.n_iters++;
            is.palette_total += r.P;
            if (h->edges_on) {
                is.edges += hv[2 * na + a];
                is.max_edges = std::max<int64_t>(is.max_edges, hv[2 * na + a]);
            } else {
                is.edges = is.max_edges = -1;
            }
            if (r.m - mi[i] <= 0) throw Error(PICASSO_EINTERNAL, "iteration coloured no vertex of an instance");
        }
        it.colored = m - m_next;
        it.ms_buckets = tm.ms(0, 1);
        it.ms_graph = tm.ms(1, 2);
        it.ms_color = tm.ms(2, 3);
        it.ms_compact = tm.ms(3, 4);
        add_iter(S, iter_edges, ell - 1, it);
        // instances with few vertices left finish in the tail kernel; the
        // others' vertices move to the front of the next vertex set
        bool gathered = false;
        // (with a schedule, once every further iteration uses its last entry)
        if (tails && (ra.n_steps == 0 || (int32_t)ell + 1 >= ra.n_steps)) {
            const int64_t kept = run_tails(h, ra, act, mi, off, ell, d_out, tp, gathered);
            m_next = kept;
        }
        if (!gathered) std::swap(h->ids, h->next_ids);
        m = m_next;
        ++ell;
    }
    tail_plan_finish(h, tp, off, n_colors, S, iter_edges);
    PCHECK_HIP(hipStreamSynchronize(st));
    for (size_t k = 0; k < iter_edges.size(); ++k) S.max_edges = std::max(S.max_edges, iter_edges[k]);
    int64_t total = 0;
    for (int32_t i = 0; i < h->nb; ++i) {
        h->istats[i].n_colors = n_colors[i];
        total += n_colors[i];
    }
    S.n_colors = total;
    S.peak_device_bytes = (int64_t)h->arena.peak;
    S.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return total;
}

__global__ void iota_kernel(int32_t *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (int32_t)i;
}

void init_ids(picasso_ctx *h, int64_t m)
{
    int32_t *ids = buf<int32_t>(h, h->ids, (size_t)std::max<int64_t>(m, 1));
    if (m > 0) {
        int64_t b = (m + 255) / 256;
        if (b > 65535 * 16) b = 65535 * 16;
        iota_kernel<<<(unsigned)b, 256, 0, h->stream>>>(ids, m);
        PCHECK_LAUNCH();
    }
}

template <typename F>
auto guarded(F &&f, decltype(f()) on_error) -> decltype(f())
{
    try {
        return f();
    } catch (const Error &e) {
        set_last_error(e.what());
        return static_cast<decltype(f())>(e.code);
    } catch (const std::bad_alloc &) {
        set_last_error("host allocation failed");
        return static_cast<decltype(f())>(PICASSO_ENOMEM);
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return on_error;
    }
}

void check_handle(picasso_handle h)
{
    if (!h) throw Error(PICASSO_EINVAL, "null handle");
    PCHECK_HIP(hipSetDevice(h->device));
}

void check_rel(int32_t rel)
{
    if (rel != PICASSO_REL_ANTICOMMUTE && rel != PICASSO_REL_QWC && rel != PICASSO_REL_COMMUTE)
        throw Error(PICASSO_EINVAL, "unknown relation");
}

void check_single(picasso_ctx *h)
{
    if (h->nb != 1) throw Error(PICASSO_EINVAL, "this call takes a single-instance handle (use picasso_color_batch)");
}

void check_color_args(double frac, double alpha, int32_t rel)
{
    if (!(frac > 0.0 && frac <= 1.0)) throw Error(PICASSO_EINVAL, "palette_frac must be in (0, 1]");
    if (!(alpha > 0.0) || !std::isfinite(alpha)) throw Error(PICASSO_EINVAL, "list_size must be > 0");
    check_rel(rel);
}

picasso_handle create_impl(int64_t n, int32_t q, const uint64_t *x, const uint64_t *z, bool device_src)
{
    if (n < 0 || n >= ((int64_t)1 << 31)) throw Error(PICASSO_EINVAL, "n must be in [0, 2^31)");
    if (q < 1 || q > 256) throw Error(PICASSO_EINVAL, "q must be in [1, 256]");
    if (n > 0 && (!x || !z)) throw Error(PICASSO_EINVAL, "null string pointer");
    const int W = (q + 63) / 64;
    if (!device_src && n > 0 && q % 64) {
        const uint64_t mask = ~((1ull << (q % 64)) - 1ull);
        for (int64_t i = 0; i < n; ++i)
            if ((x[i * W + W - 1] | z[i * W + W - 1]) & mask) throw Error(PICASSO_EINVAL, "padding bits set");
    }
    auto *h = new picasso_ctx();
    try {
        PCHECK_HIP(hipGetDevice(&h->device));
        PCHECK_HIP(hipStreamCreateWithFlags(&h->own_stream, hipStreamNonBlocking));
        h->stream = h->own_stream;
        h->n = n;
        h->q = q;
        h->W = W;
        h->nb = 1;
        h->inst_n.assign(1, n);
        h->inst_base.assign(1, 0);
        h->inst_q.assign(1, q);
        const size_t bytes = (size_t)std::max<int64_t>(n, 1) * W * sizeof(uint64_t);
        uint64_t *dx = static_cast<uint64_t *>(h->arena.ensure(h->x, bytes));
        uint64_t *dz = static_cast<uint64_t *>(h->arena.ensure(h->z, bytes));
        const size_t cb = (size_t)n * W * sizeof(uint64_t);
        if (cb) {
            const hipMemcpyKind kind = device_src ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
            PCHECK_HIP(hipMemcpyAsync(dx, x, cb, kind, h->stream));
            PCHECK_HIP(hipMemcpyAsync(dz, z, cb, kind, h->stream));
        }
        uint64_t *dxz = static_cast<uint64_t *>(h->arena.ensure(h->xz, 2 * bytes));
        launch_interleave(dx, dz, n, W, dxz, h->stream);
        if (device_src && n > 0) {
            int32_t *bad = buf<int32_t>(h, h->scalars, 16);
            launch_fill_i32(bad, 1, 0, h->stream);
            launch_check_padding(dx, dz, n, q, bad, h->stream);
            if (read_scalar(h, bad)) throw Error(PICASSO_EINVAL, "padding bits set");
        }
        PCHECK_HIP(hipStreamSynchronize(h->stream));
    } catch (...) {
        picasso_destroy(h);
        throw;
    }
    return h;
}

// Instances packed back to back, each row widened to the words of the
// largest q (zero words above an instance's own q change neither relation).
picasso_handle create_batch_impl(int32_t count, const int64_t *ns, const int32_t *qs, const uint64_t *x,
                                 const uint64_t *z)
{
    if (count < 1) throw Error(PICASSO_EINVAL, "count must be >= 1");
    if (!ns || !qs) throw Error(PICASSO_EINVAL, "null sizes");
    int64_t total = 0;
    int32_t qmax = 1;
    for (int32_t i = 0; i < count; ++i) {
        if (ns[i] < 0 || ns[i] >= ((int64_t)1 << 31)) throw Error(PICASSO_EINVAL, "n must be in [0, 2^31)");
        if (qs[i] < 1 || qs[i] > 256) throw Error(PICASSO_EINVAL, "q must be in [1, 256]");
        total += ns[i];
        qmax = std::max(qmax, qs[i]);
    }
    if (total >= ((int64_t)1 << 31)) throw Error(PICASSO_EINVAL, "total strings must be < 2^31");
    if (total > 0 && (!x || !z)) throw Error(PICASSO_EINVAL, "null string pointer");
    const int W = (qmax + 63) / 64;
    std::vector<uint64_t> px((size_t)total * W, 0ull), pz((size_t)total * W, 0ull);
    std::vector<int64_t> base((size_t)count);
    int64_t row = 0, word = 0;
    for (int32_t i = 0; i < count; ++i) {
        const int Wi = (qs[i] + 63) / 64;
        const uint64_t mask = qs[i] % 64 ? ~((1ull << (qs[i] % 64)) - 1ull) : 0ull;
        base[i] = row;
        for (int64_t r = 0; r < ns[i]; ++r, ++row, word += Wi) {
            if ((x[word + Wi - 1] | z[word + Wi - 1]) & mask)
                throw Error(PICASSO_EINVAL, "padding bits set in instance " + std::to_string(i));
            for (int w = 0; w < Wi; ++w) {
                px[(size_t)row * W + w] = x[word + w];
                pz[(size_t)row * W + w] = z[word + w];
            }
        }
    }
    picasso_handle h = create_impl(total, qmax, px.data(), pz.data(), false);
    h->nb = count;
    h->inst_n.assign(ns, ns + count);
    h->inst_base = base;
    h->inst_q.assign(qs, qs + count);
    return h;
}

}  // namespace

extern "C" {

const char *picasso_last_error(void) { return g_last_error.c_str(); }

picasso_handle picasso_create(int64_t n, int32_t q, const uint64_t *x_words, const uint64_t *z_words)
{
    try {
        return create_impl(n, q, x_words, z_words, false);
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return nullptr;
    }
}

picasso_handle picasso_create_device(int64_t n, int32_t q, const uint64_t *x_words, const uint64_t *z_words)
{
    try {
        return create_impl(n, q, x_words, z_words, true);
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return nullptr;
    }
}

picasso_handle picasso_create_batch(int32_t count, const int64_t *ns, const int32_t *qs, const uint64_t *x_words,
                                    const uint64_t *z_words)
{
    try {
        return create_batch_impl(count, ns, qs, x_words, z_words);
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return nullptr;
    }
}

void picasso_destroy(picasso_handle h)
{
    if (!h) return;
    (void)hipSetDevice(h->device);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    DevBuf *all[] = {&h->x,       &h->z,       &h->xz,        &h->ids,     &h->next_ids, &h->lists,   &h->prio,     &h->bcnt,
                     &h->bstart,  &h->bmem,     &h->bslot,   &h->pos_of,   &h->bent, &h->tmp_mem, &h->tmp_slot, &h->tiles,
                     &h->words,   &h->tile_off, &h->rb_off,  &h->R,        &h->D,       &h->nslow,    &h->slow,
                     &h->seg,      &h->seg_off,  &h->deg,      &h->rowptr, &h->adj,      &h->col,     &h->blk,      &h->fre,
                     &h->nblk,    &h->st,       &h->rdy,     &h->jp_prog, &h->dflag, &h->wl,       &h->flags,   &h->pos,      &h->used,
                     &h->scan_tmp, &h->bx,      &h->bz,      &h->tile_bucket,
                     &h->scalars, &h->out_colors, &h->judge_out, &h->inst,    &h->vinst,    &h->loff,    &h->binst,    &h->inst_out, &h->tail_recs,
                     &h->tail_table, &h->tail_outs, &h->tail_iters, &h->tail_ranges, &h->tail_ids, &h->wake_at,
                     &h->hits,    &h->csr_flag, &h->rkey,  &h->dyn_hist, &h->dyn_sstar, &h->dyn_cut,
                     &h->rx_k32a, &h->rx_k32b, &h->rx_va, &h->rx_vb,   &h->rx_tmp,  &h->rx_tr,   &h->rx_at,
                     &h->rx_cka,  &h->rx_ckb,  &h->rx_cva, &h->rx_cvb};
    for (DevBuf *b : all) h->arena.release(*b);
    if (h->tail_stream) (void)hipStreamSynchronize(h->tail_stream);
    if (h->tail_ready) (void)hipEventDestroy(h->tail_ready);
    if (h->tail_done) (void)hipEventDestroy(h->tail_done);
    if (h->tail_stream) (void)hipStreamDestroy(h->tail_stream);
    if (h->own_stream) (void)hipStreamDestroy(h->own_stream);
    delete h;
}

int32_t picasso_set_option(picasso_handle h, int32_t key, int64_t value)
{
    return guarded(
        [&]() -> int32_t {
            check_handle(h);
            switch (key) {
                case PICASSO_OPT_MEM_BUDGET:
                    if (value < 0) throw Error(PICASSO_EINVAL, "budget must be >= 0");
                    h->mem_budget = value;
                    break;
                case PICASSO_OPT_PAIR_PATH:
                    if (value < 0 || value > 2) throw Error(PICASSO_EINVAL, "unknown pair path");
                    h->pair_path = (int32_t)value;
                    break;
                case PICASSO_OPT_FIXED_T:
                    if (value < 0 || value > PICASSO_MAX_T) throw Error(PICASSO_EINVAL, "fixed T out of range");
                    h->fixed_T = (int32_t)value;
                    break;
                case PICASSO_OPT_STREAM:
                    h->stream = value ? reinterpret_cast<hipStream_t>(value) : h->own_stream;
                    break;
                case PICASSO_OPT_TIMING:
                    h->timing = value != 0;
                    break;
                case PICASSO_OPT_JP_BATCH:
                    if (value < 1 || value > 1024) throw Error(PICASSO_EINVAL, "rounds per check must be in [1, 1024]");
                    h->jp_batch = (int32_t)value;
                    break;
                case PICASSO_OPT_GRAPH:
                    h->use_graph = value != 0;
                    break;
                case PICASSO_OPT_TAIL:
                    h->use_tail = value != 0;
                    break;
                case PICASSO_OPT_BUCKET_BUILD:
                    if (value < 0 || value > 2) throw Error(PICASSO_EINVAL, "bucket build is 0, 1 or 2");
                    h->bucket_build = (int32_t)value;
                    break;
                case PICASSO_OPT_EDGES:
                    if (value != 0 && value != 1) throw Error(PICASSO_EINVAL, "the edges option is 0 or 1");
                    h->edges_on = (int32_t)value;
                    break;
                case PICASSO_OPT_COLOURER:
                    if (value != PICASSO_COLOURER_STATIC && value != PICASSO_COLOURER_DYNAMIC)
                        throw Error(PICASSO_EINVAL, "unknown colourer");
                    h->colourer = (int32_t)value;
                    break;
                case PICASSO_OPT_DYN_DIVISOR:
                    if (value < 1 || value > (1 << 20)) throw Error(PICASSO_EINVAL, "divisor must be in [1, 2^20]");
                    h->dyn_divisor = (int32_t)value;
                    break;
                case PICASSO_OPT_CSR_SIZING:
                    if (value < 0 || value > 2) throw Error(PICASSO_EINVAL, "CSR sizing is 0, 1 or 2");
                    h->csr_sizing = (int32_t)value;
                    break;
                case PICASSO_OPT_LEARNED_JUDGE:
                    if (value != 0 && value != 1) throw Error(PICASSO_EINVAL, "the judge option is 0 or 1");
                    h->judge = (int32_t)value;
                    break;
                case PICASSO_OPT_MFMA_CAP:
                    if (value < -1 || value > 4096) throw Error(PICASSO_EINVAL, "MFMA bucket cap must be in [-1, 4096]");
                    h->mfma_cap = value;
                    break;
                default:
                    throw Error(PICASSO_EINVAL, "unknown option");
            }
            return PICASSO_OK;
        },
        PICASSO_EINTERNAL);
}

int64_t picasso_color_device(picasso_handle h, uint64_t seed, double palette_frac, double list_size,
                             int32_t relation, int32_t *out_colors)
{
    return guarded(
        [&]() -> int64_t {
            check_handle(h);
            check_single(h);
            check_color_args(palette_frac, list_size, relation);
            if (h->n > 0 && !out_colors) throw Error(PICASSO_EINVAL, "null output");
            if (h->n == 0) {
                std::memset(&h->stats, 0, sizeof(h->stats));
                return 0;
            }
            RunArgs ra{&seed, &palette_frac, &list_size, &relation};
            int64_t nc = 0;
            return color_all(h, ra, out_colors, &nc);
        },
        PICASSO_EINTERNAL);
}

int64_t picasso_color(picasso_handle h, uint64_t seed, double palette_frac, double list_size, int32_t relation,
                      int32_t *out_colors)
{
    return guarded(
        [&]() -> int64_t {
            check_handle(h);
            check_single(h);
            check_color_args(palette_frac, list_size, relation);
            if (h->n > 0 && !out_colors) throw Error(PICASSO_EINVAL, "null output");
            if (h->n == 0) {
                std::memset(&h->stats, 0, sizeof(h->stats));
                return 0;
            }
            int32_t *d_out = buf<int32_t>(h, h->out_colors, (size_t)h->n);
            RunArgs ra{&seed, &palette_frac, &list_size, &relation};
            int64_t n_colors = 0;
            const int64_t nc = color_all(h, ra, d_out, &n_colors);
            const auto t0 = std::chrono::steady_clock::now();
            download(h, out_colors, d_out, (size_t)h->n * sizeof(int32_t));
            h->stats.ms_total +=
                std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            return nc;
        },
        PICASSO_EINTERNAL);
}

static int64_t color_batch_impl(picasso_handle h, const uint64_t *seeds, const double *palette_fracs,
                                const double *list_sizes, const int32_t *relations, int32_t *out_colors,
                                int64_t *out_n_colors, bool device_out)
{
    return guarded(
        [&]() -> int64_t {
            check_handle(h);
            if (!seeds || !palette_fracs || !list_sizes || !relations || !out_n_colors)
                throw Error(PICASSO_EINVAL, "null argument");
            for (int32_t i = 0; i < h->nb; ++i) check_color_args(palette_fracs[i], list_sizes[i], relations[i]);
            if (h->n > 0 && !out_colors) throw Error(PICASSO_EINVAL, "null output");
            if (h->n == 0) {
                std::memset(&h->stats, 0, sizeof(h->stats));
                h->istats.assign((size_t)h->nb, picasso_instance_stats{});
                for (int32_t i = 0; i < h->nb; ++i) out_n_colors[i] = 0;
                return 0;
            }
            int32_t *d_out = device_out ? out_colors : buf<int32_t>(h, h->out_colors, (size_t)h->n);
            RunArgs ra{seeds, palette_fracs, list_sizes, relations};
            const int64_t nc = color_all(h, ra, d_out, out_n_colors);
            if (!device_out) download(h, out_colors, d_out, (size_t)h->n * sizeof(int32_t));
            return nc;
        },
        PICASSO_EINTERNAL);
}

int64_t picasso_color_batch(picasso_handle h, const uint64_t *seeds, const double *palette_fracs,
                            const double *list_sizes, const int32_t *relations, int32_t *out_colors,
                            int64_t *out_n_colors)
{
    return color_batch_impl(h, seeds, palette_fracs, list_sizes, relations, out_colors, out_n_colors, false);
}

int64_t picasso_color_batch_device(picasso_handle h, const uint64_t *seeds, const double *palette_fracs,
                                   const double *list_sizes, const int32_t *relations, int32_t *out_colors,
                                   int64_t *out_n_colors)
{
    return color_batch_impl(h, seeds, palette_fracs, list_sizes, relations, out_colors, out_n_colors, true);
}

int32_t picasso_get_instance_stats(picasso_handle h, int32_t count, picasso_instance_stats *out)
{
    return guarded(
        [&]() -> int32_t {
            if (!h) throw Error(PICASSO_EINVAL, "null handle");
            if (count < 0 || count > h->nb || (count > 0 && !out)) throw Error(PICASSO_EINVAL, "bad count or output");
            for (int32_t i = 0; i < count; ++i)
                out[i] = i < (int32_t)h->istats.size() ? h->istats[i] : picasso_instance_stats{};
            return h->nb;
        },
        PICASSO_EINTERNAL);
}

int32_t picasso_get_stats(picasso_handle h, picasso_stats *out)
{
    return guarded(
        [&]() -> int32_t {
            if (!h || !out) throw Error(PICASSO_EINVAL, "null argument");
            *out = h->stats;
            return PICASSO_OK;
        },
        PICASSO_EINTERNAL);
}

static void check_subset(picasso_ctx *h, int64_t m, const int32_t *ids, int64_t P, int32_t T)
{
    if (m < 0 || m > h->n) throw Error(PICASSO_EINVAL, "m out of range");
    if (m > 0 && !ids) throw Error(PICASSO_EINVAL, "null ids");
    if (P < 1 || P > INT32_MAX) throw Error(PICASSO_EINVAL, "P out of range");
    if (T < 1 || T > P || T > PICASSO_MAX_T) throw Error(PICASSO_EINVAL, "T out of range");
    for (int64_t i = 0; i < m; ++i) {
        if (ids[i] < 0 || ids[i] >= h->n) throw Error(PICASSO_EINVAL, "id out of range");
        if (i && ids[i] <= ids[i - 1]) throw Error(PICASSO_EINVAL, "ids must be strictly ascending");
    }
}

int32_t picasso_sample_lists(picasso_handle h, uint64_t seed, int32_t ell, int64_t m, const int32_t *ids, int64_t P,
                             int32_t T, uint32_t *out_lists, uint64_t *out_prio)
{
    return guarded(
        [&]() -> int32_t {
            check_handle(h);
            check_single(h);
            check_subset(h, m, ids, P, T);
            if (m > 0 && !out_lists) throw Error(PICASSO_EINVAL, "null output");
            if (m == 0) return PICASSO_OK;
            int32_t *d_ids = buf<int32_t>(h, h->ids, (size_t)m);
            upload(h, d_ids, ids, (size_t)m * sizeof(int32_t));
            uint32_t *lists = buf<uint32_t>(h, h->lists, (size_t)m * T);
            uint64_t *prio = buf<uint64_t>(h, h->prio, (size_t)m);
            const Batch b = single_instance(h, seed, m, P, T, PICASSO_REL_ANTICOMMUTE);
            launch_sample_lists(b, (uint32_t)ell, m, d_ids, T, lists, prio, h->stream);
            download(h, out_lists, lists, (size_t)m * T * sizeof(uint32_t));
            if (out_prio) download(h, out_prio, prio, (size_t)m * sizeof(uint64_t));
            return PICASSO_OK;
        },
        PICASSO_EINTERNAL);
}

int64_t picasso_conflict_graph(picasso_handle h, uint64_t seed, int32_t ell, int64_t m, const int32_t *ids, int64_t P,
                               int32_t T, int32_t relation, int64_t *out_rowptr, int32_t *out_adj, int64_t adj_cap)
{
    return guarded(
        [&]() -> int64_t {
            check_handle(h);
            check_single(h);
            check_subset(h, m, ids, P, T);
            check_rel(relation);
            if (m == 0) {
                if (out_rowptr) out_rowptr[0] = 0;
                return 0;
            }
            int32_t *d_ids = buf<int32_t>(h, h->ids, (size_t)m);
            upload(h, d_ids, ids, (size_t)m * sizeof(int32_t));
            Batch b = single_instance(h, seed, m, P, T, relation);
            const BucketInfo bi = build_lists_and_buckets(h, b, (uint32_t)ell, m, d_ids, m * T, P, T);
            // above the memory budget the CSR is counted here and written in chunks below
            const int64_t edges =
                build_conflict_graph(h, b, m, m * T, P, T, 1 << relation, bi, nullptr, nullptr, nullptr, false);
            const int64_t total = 2 * edges;
            const bool whole = h->mem_budget <= 0 || total * (int64_t)sizeof(int32_t) <= h->mem_budget;
            std::vector<int64_t> rp;
            int64_t *rowptr = out_rowptr;
            if (!rowptr && out_adj && total <= adj_cap && !whole) {
                rp.resize((size_t)m + 1);
                rowptr = rp.data();
            }
            if (rowptr) download(h, rowptr, h->rowptr.p, (size_t)(m + 1) * sizeof(int64_t));
            if (out_adj && total <= adj_cap) {
                if (whole)
                    download(h, out_adj, h->adj.p, (size_t)total * sizeof(int32_t));
                else
                    fill_csr_chunks(h, b, m, P, bi, rowptr, out_adj);
            }
            return edges;
        },
        PICASSO_EINTERNAL);
}

int64_t picasso_list_color_csr(picasso_handle h, int64_t m, const uint64_t *prio, const uint32_t *lists, int32_t T,
                               int64_t P, const int64_t *rowptr, const int32_t *adj, int32_t *out_col)
{
    return guarded(
        [&]() -> int64_t {
            check_handle(h);
            check_single(h);
            if (m < 0 || m >= ((int64_t)1 << 31)) throw Error(PICASSO_EINVAL, "m out of range");
            if (T < 1 || T > PICASSO_MAX_T || P < 1 || T > P) throw Error(PICASSO_EINVAL, "bad T or P");
            if (m == 0) return 0;
            if (!prio || !lists || !rowptr || !out_col) throw Error(PICASSO_EINVAL, "null argument");
            const int64_t total = rowptr[m];
            if (rowptr[0] != 0 || total < 0 || (total > 0 && !adj)) throw Error(PICASSO_EINVAL, "bad CSR");
            for (int64_t i = 0; i < m; ++i)
                if (rowptr[i + 1] < rowptr[i]) throw Error(PICASSO_EINVAL, "bad CSR");
            for (int64_t e = 0; e < total; ++e)
                if (adj[e] < 0 || adj[e] >= m) throw Error(PICASSO_EINVAL, "CSR index out of range");
            for (int64_t e = 0; e < m * T; ++e)
                if (lists[e] >= (uint64_t)P) throw Error(PICASSO_EINVAL, "list colour out of range");
            for (int64_t i = 0; i < m; ++i)
                for (int k = 1; k < T; ++k)
                    if (lists[i * T + k] <= lists[i * T + k - 1]) throw Error(PICASSO_EINVAL, "list rows must be sorted");
            upload(h, buf<uint64_t>(h, h->prio, (size_t)m), prio, (size_t)m * sizeof(uint64_t));
            upload(h, buf<uint32_t>(h, h->lists, (size_t)m * T), lists, (size_t)m * T * sizeof(uint32_t));
            int64_t *d_rowptr = buf<int64_t>(h, h->rowptr, (size_t)m + 1);
            int32_t *d_adj = buf<int32_t>(h, h->adj, (size_t)std::max<int64_t>(total, 1));
            upload(h, d_rowptr, rowptr, (size_t)(m + 1) * sizeof(int64_t));
            upload(h, d_adj, adj, (size_t)total * sizeof(int32_t));
            Batch b = single_instance(h, 0, m, P, T, PICASSO_REL_ANTICOMMUTE);
            const BucketInfo bi = buckets_from_lists(h, b, m, m * T, P);
            uint64_t *R = buf<uint64_t>(h, h->R, (size_t)std::max<int64_t>(bi.words, 1));
            launch_fill_u64(R, bi.words, 0ull, h->stream);
            launch_csr_to_relation(m, d_rowptr, d_adj, static_cast<const uint32_t *>(h->lists.p), b.loff,
                                   static_cast<const int64_t *>(h->pos_of.p), static_cast<const int64_t *>(h->bstart.p),
                                   static_cast<const int64_t *>(h->rb_off.p), R, h->stream);
            color_buckets(h, b, m, m * T, P, T, bi);
            download(h, out_col, h->col.p, (size_t)m * sizeof(int32_t));
            int64_t colored = 0;
            for (int64_t i = 0; i < m; ++i) colored += out_col[i] >= 0;
            return colored;
        },
        PICASSO_EINTERNAL);
}

int32_t picasso_features(picasso_handle h, uint64_t seed, int32_t ell, int64_t m, const int32_t *ids,
                         int32_t relation, double *out)
{
    return guarded(
        [&]() -> int32_t {
            check_handle(h);
            check_single(h);
            check_rel(relation);
            if (!out) throw Error(PICASSO_EINVAL, "null output");
            check_subset(h, m, ids, 1, 1);
            int32_t *d_ids = buf<int32_t>(h, h->ids, (size_t)std::max<int64_t>(m, 1));
            upload(h, d_ids, ids, (size_t)m * sizeof(int32_t));
            device_features(h, seed, (uint32_t)ell, m, d_ids, h->q, relation, out);
            return PICASSO_OK;
        },
        PICASSO_EINTERNAL);
}

picasso_mlp picasso_mlp_create(const float *params, uint64_t seed)
{
    auto *c = new picasso_mlp_ctx();
    try {
        PCHECK_HIP(hipGetDevice(&c->device));
        PCHECK_HIP(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
        std::vector<float> init(kMlpParams, 0.0f);
        if (params) {
            std::memcpy(init.data(), params, sizeof(float) * kMlpParams);
        } else {
            // He-scaled normal weights, zero biases, from a seeded std generator
            std::mt19937_64 gen(seed);
            std::normal_distribution<double> nd(0.0, 1.0);
            const int layers[3][3] = {{0, kMlpHidden * kMlpIn, kMlpIn},
                                      {kMlpHidden * kMlpIn + kMlpHidden, kMlpHidden * kMlpHidden, kMlpHidden},
                                      {kMlpHidden * kMlpIn + 2 * kMlpHidden + kMlpHidden * kMlpHidden,
                                       kMlpOut * kMlpHidden, kMlpHidden}};
            for (const auto &L : layers) {
                const double sd = std::sqrt(2.0 / L[2]);
                for (int i = 0; i < L[1]; ++i) init[L[0] + i] = (float)(nd(gen) * sd);
            }
        }
        float *dp = mbuf<float>(c, c->params, kMlpParams);
        PCHECK_HIP(hipMemcpyAsync(dp, init.data(), sizeof(float) * kMlpParams, hipMemcpyHostToDevice, c->stream));
        float *m1 = mbuf<float>(c, c->m1, kMlpParams);
        float *m2 = mbuf<float>(c, c->m2, kMlpParams);
        PCHECK_HIP(hipMemsetAsync(m1, 0, sizeof(float) * kMlpParams, c->stream));
        PCHECK_HIP(hipMemsetAsync(m2, 0, sizeof(float) * kMlpParams, c->stream));
        PCHECK_HIP(hipStreamSynchronize(c->stream));
    } catch (const std::exception &e) {
        set_last_error(e.what());
        picasso_mlp_destroy(c);
        return nullptr;
    }
    return c;
}

void picasso_mlp_destroy(picasso_mlp c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    DevBuf *all[] = {&c->params, &c->m1, &c->m2, &c->raw, &c->target, &c->out, &c->keep, &c->row_loss, &c->grad, &c->fa};
    for (DevBuf *b : all) c->arena.release(*b);
    if (c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

static void check_mlp(picasso_mlp c)
{
    if (!c) throw Error(PICASSO_EINVAL, "null network");
    PCHECK_HIP(hipSetDevice(c->device));
}

int32_t picasso_mlp_get_params(picasso_mlp c, float *out)
{
    return guarded(
        [&]() -> int32_t {
            check_mlp(c);
            if (!out) throw Error(PICASSO_EINVAL, "null output");
            PCHECK_HIP(hipMemcpyAsync(out, c->params.p, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost, c->stream));
            PCHECK_HIP(hipStreamSynchronize(c->stream));
            return PICASSO_OK;
        },
        PICASSO_EINTERNAL);
}

int32_t picasso_mlp_set_params(picasso_mlp c, const float *in)
{
    return guarded(
        [&]() -> int32_t {
            check_mlp(c);
            if (!in) throw Error(PICASSO_EINVAL, "null input");
            PCHECK_HIP(hipMemcpyAsync(c->params.p, in, sizeof(float) * kMlpParams, hipMemcpyHostToDevice, c->stream));
            PCHECK_HIP(hipMemsetAsync(c->m1.p, 0, sizeof(float) * kMlpParams, c->stream));
            PCHECK_HIP(hipMemsetAsync(c->m2.p, 0, sizeof(float) * kMlpParams, c->stream));
            PCHECK_HIP(hipStreamSynchronize(c->stream));
            c->step = 0;
            return PICASSO_OK;
        },
        PICASSO_EINTERNAL);
}

int32_t picasso_mlp_forward(picasso_mlp c, const float *features, int32_t B, float *out)
{
    return guarded(
        [&]() -> int32_t {
            check_mlp(c);
            if (B < 0 || (B > 0 && (!features || !out))) throw Error(PICASSO_EINVAL, "bad batch");
            if (B == 0) return PICASSO_OK;
            float *d_raw = mbuf<float>(c, c->raw, (size_t)B * kMlpIn);
            float *d_out = mbuf<float>(c, c->out, (size_t)B * kMlpOut);
            PCHECK_HIP(hipMemcpyAsync(d_raw, features, sizeof(float) * B * kMlpIn, hipMemcpyHostToDevice, c->stream));
            launch_mlp_rows(static_cast<const float *>(c->params.p), d_raw, B, d_out, nullptr, nullptr, nullptr,
                            c->stream);
            PCHECK_HIP(hipMemcpyAsync(out, d_out, sizeof(float) * B * kMlpOut, hipMemcpyDeviceToHost, c->stream));
            PCHECK_HIP(hipStreamSynchronize(c->stream));
            return PICASSO_OK;
        },
        PICASSO_EINTERNAL);
}

// Forward with training state, then the gradient; returns the batch loss.
static float mlp_gradient_impl(picasso_mlp c, const float *features, const float *target, int32_t B)
{
    if (B <= 0 || !features || !target) throw Error(PICASSO_EINVAL, "bad batch");
    float *d_raw = mbuf<float>(c, c->raw, (size_t)B * kMlpIn);
    float *d_t = mbuf<float>(c, c->target, (size_t)B * kMlpOut);
    float *d_keep = mbuf<float>(c, c->keep, (size_t)B * kMlpKeep);
    float *d_loss = mbuf<float>(c, c->row_loss, (size_t)B);
    float *d_grad = mbuf<float>(c, c->grad, kMlpParams);
    PCHECK_HIP(hipMemcpyAsync(d_raw, features, sizeof(float) * B * kMlpIn, hipMemcpyHostToDevice, c->stream));
    PCHECK_HIP(hipMemcpyAsync(d_t, target, sizeof(float) * B * kMlpOut, hipMemcpyHostToDevice, c->stream));
    launch_mlp_rows(static_cast<const float *>(c->params.p), d_raw, B, nullptr, d_t, d_keep, d_loss, c->stream);
    launch_mlp_grad(d_keep, B, d_grad, c->stream);
    std::vector<float> rl(B);
    PCHECK_HIP(hipMemcpyAsync(rl.data(), d_loss, sizeof(float) * B, hipMemcpyDeviceToHost, c->stream));
    PCHECK_HIP(hipStreamSynchronize(c->stream));
    double loss = 0.0;
    for (float v : rl) loss += v;
    return (float)loss;
}

int32_t picasso_mlp_gradient(picasso_mlp c, const float *features, const float *target, int32_t B, float *grad,
                             float *loss)
{
    return guarded(
        [&]() -> int32_t {
            check_mlp(c);
            const float l = mlp_gradient_impl(c, features, target, B);
            if (loss) *loss = l;
            if (grad) {
                PCHECK_HIP(hipMemcpyAsync(grad, c->grad.p, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost, c->stream));
                PCHECK_HIP(hipStreamSynchronize(c->stream));
            }
            return PICASSO_OK;
        },
        PICASSO_EINTERNAL);
}

int32_t picasso_mlp_train_step(picasso_mlp c, const float *features, const float *target, int32_t B, float lr,
                               float *loss)
{
    return guarded(
        [&]() -> int32_t {
            check_mlp(c);
            if (!(lr > 0.0f)) throw Error(PICASSO_EINVAL, "learning rate must be > 0");
            const float l = mlp_gradient_impl(c, features, target, B);
            ++c->step;
            launch_adam(static_cast<float *>(c->params.p), static_cast<const float *>(c->grad.p),
                        static_cast<float *>(c->m1.p), static_cast<float *>(c->m2.p), lr, 0.9f, 0.999f, 1e-8f,
                        c->step, c->stream);
            PCHECK_HIP(hipStreamSynchronize(c->stream));
            if (loss) *loss = l;
            return PICASSO_OK;
        },
        PICASSO_EINTERNAL);
}

int64_t picasso_color_schedule(picasso_handle h, uint64_t seed, const double *palette_fracs, const double *list_sizes,
                               int32_t count, int32_t relation, int32_t *out_colors)
{
    return guarded(
        [&]() -> int64_t {
            check_handle(h);
            check_single(h);
            if (count < 1 || !palette_fracs || !list_sizes) throw Error(PICASSO_EINVAL, "empty schedule");
            for (int32_t k = 0; k < count; ++k) check_color_args(palette_fracs[k], list_sizes[k], relation);
            if (h->n > 0 && !out_colors) throw Error(PICASSO_EINVAL, "null output");
            if (h->n == 0) {
                std::memset(&h->stats, 0, sizeof(h->stats));
                return 0;
            }
            int32_t *d_out = buf<int32_t>(h, h->out_colors, (size_t)h->n);
            RunArgs ra{&seed, &palette_fracs[count - 1], &list_sizes[count - 1], &relation};
            ra.step_f = palette_fracs;
            ra.step_a = list_sizes;
            ra.n_steps = count;
            int64_t n_colors = 0;
            const int64_t nc = color_all(h, ra, d_out, &n_colors);
            download(h, out_colors, d_out, (size_t)h->n * sizeof(int32_t));
            return nc;
        },
        PICASSO_EINTERNAL);
}

int64_t picasso_color_learned(picasso_handle h, uint64_t seed, picasso_mlp mlp, double beta, int32_t relation,
                              int32_t *out_colors, float *out_schedule, int32_t max_sched)
{
    return guarded(
        [&]() -> int64_t {
            check_handle(h);
            check_single(h);
            check_rel(relation);
            if (!(beta >= 0.0 && beta <= 1.0)) throw Error(PICASSO_EINVAL, "beta must be in [0, 1]");
            if (!mlp) throw Error(PICASSO_EINVAL, "null network");
            if (h->n > 0 && !out_colors) throw Error(PICASSO_EINVAL, "null output");
            if (mlp->device != h->device) throw Error(PICASSO_EINVAL, "network and handle on different devices");
            if (h->n == 0) {
                std::memset(&h->stats, 0, sizeof(h->stats));
                return 0;
            }
            int32_t *d_out = buf<int32_t>(h, h->out_colors, (size_t)h->n);
            const double f0 = kFixedFrac, a0 = kFixedAlpha;
            RunArgs ra{&seed, &f0, &a0, &relation, mlp, out_schedule, max_sched};
            ra.beta = beta;
            int64_t n_colors = 0;
            const int64_t nc = color_all(h, ra, d_out, &n_colors);
            if (!h->judge) {
                download(h, out_colors, d_out, (size_t)h->n * sizeof(int32_t));
                return nc;
            }
            // judge: the fixed-parameter colouring of the same strings and
            // seed; the network's result is kept unless the fixed one uses
            // fewer colours
            const picasso_stats learned_stats = h->stats;
            const std::vector<picasso_instance_stats> learned_istats = h->istats;
            int32_t *d_fixed = buf<int32_t>(h, h->judge_out, (size_t)h->n);
            RunArgs rf{&seed, &f0, &a0, &relation};
            int64_t nf_colors = 0;
            const int64_t nf = color_all(h, rf, d_fixed, &nf_colors);
            const double ms_fixed = h->stats.ms_total;
            const int64_t peak = std::max<int64_t>(learned_stats.peak_device_bytes, h->stats.peak_device_bytes);
            if (nf < nc) {
                download(h, out_colors, d_fixed, (size_t)h->n * sizeof(int32_t));
                h->stats.judged = PICASSO_JUDGE_FIXED;
                h->stats.peak_device_bytes = peak;
                h->stats.ms_total += learned_stats.ms_total;
                return nf;
            }
            download(h, out_colors, d_out, (size_t)h->n * sizeof(int32_t));
            h->stats = learned_stats;
            h->istats = learned_istats;
            h->stats.judged = PICASSO_JUDGE_LEARNED;
            h->stats.peak_device_bytes = peak;
            h->stats.ms_total += ms_fixed;
            return nc;
        },
        PICASSO_EINTERNAL);
}

}  // extern "C"
