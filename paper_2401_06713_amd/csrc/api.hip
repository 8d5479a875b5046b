// Host driver and C ABI (Alg. 1 iteration loop around the device steps).
//
// Per iteration: (P, T) in host double arithmetic -> lists and priorities ->
// colour buckets (count, scan, scatter) -> pair count pass -> row-pointer
// scan -> pair fill pass into the CSR -> list colouring -> write global
// colours, compact the uncoloured vertices (ascending ids) -> next palette.
// The only device->host traffic inside the loop is a few scalars.
#include <chrono>
#include <cmath>
#include <cstring>
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
    int64_t n = 0;
    int32_t q = 0, W = 0;
    int device = 0;
    hipStream_t own_stream = nullptr;
    hipStream_t stream = nullptr;
    int64_t mem_budget = 0;
    int32_t pair_path = PICASSO_PATH_AUTO;
    int32_t fixed_T = 0;
    int32_t timing = 0;
    Arena arena;
    DevBuf x, z;
    // iteration buffers
    DevBuf ids, next_ids, lists, prio, bcnt, bstart, bmem, bslot, deg, rowptr, adj, cursor32, col, cursor64, forbid,
        flags, pos, used, scan_tmp, scalars, out_colors;
    picasso_stats stats;
};

namespace {

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

// Lists, priorities and buckets of one iteration.  Returns pair tests.
int64_t build_lists_and_buckets(picasso_ctx *h, uint64_t seed, uint32_t ell, int64_t m, const int32_t *d_ids,
                                int64_t P, int32_t T)
{
    hipStream_t st = h->stream;
    uint32_t *lists = buf<uint32_t>(h, h->lists, (size_t)m * T);
    uint64_t *prio = buf<uint64_t>(h, h->prio, (size_t)m);
    launch_sample_lists(seed, ell, m, d_ids, P, T, lists, prio, st);
    uint32_t *bcnt = buf<uint32_t>(h, h->bcnt, (size_t)P);
    int64_t *bstart = buf<int64_t>(h, h->bstart, (size_t)P + 1);
    unsigned long long *sc = buf<unsigned long long>(h, h->scalars, 8);
    launch_fill_u32(bcnt, P, 0u, st);
    launch_fill_u32(reinterpret_cast<uint32_t *>(sc), 16, 0u, st);
    launch_bucket_count(lists, m * T, bcnt, st);
    launch_bucket_pairs(bcnt, P, sc + 0, st);
    void *tmp = h->arena.ensure(h->scan_tmp, scan_tmp_bytes(std::max<int64_t>(P, m)));
    exclusive_scan_u32_to_i64(bcnt, bstart, P, true, tmp, st);
    launch_fill_u32(bcnt, P, 0u, st);
    uint32_t *bmem = buf<uint32_t>(h, h->bmem, (size_t)m * T);
    uint8_t *bslot = buf<uint8_t>(h, h->bslot, (size_t)m * T);
    launch_bucket_scatter(lists, m, T, bstart, bcnt, bmem, bslot, st);
    return (int64_t)read_scalar(h, sc + 0);
}

PairArgs pair_args(picasso_ctx *h, int64_t m, int64_t P, int32_t T, int32_t rel)
{
    PairArgs a{};
    a.bstart = static_cast<const int64_t *>(h->bstart.p);
    a.bmem = static_cast<const uint32_t *>(h->bmem.p);
    a.bslot = static_cast<const uint8_t *>(h->bslot.p);
    a.P = P;
    a.ids = static_cast<const int32_t *>(h->ids.p);
    a.x = static_cast<const uint64_t *>(h->x.p);
    a.z = static_cast<const uint64_t *>(h->z.p);
    a.W = h->W;
    a.lists = static_cast<const uint32_t *>(h->lists.p);
    a.T = T;
    a.relation = rel;
    a.m = m;
    return a;
}

// Count pass, scan, fill pass.  Returns |E_c|; the CSR is in h->rowptr/adj.
int64_t build_conflict_graph(picasso_ctx *h, int64_t m, int64_t P, int32_t T, int32_t rel, double *ms_count,
                             double *ms_fill)
{
    hipStream_t st = h->stream;
    Timer tm(h);
    PairArgs a = pair_args(h, m, P, T, rel);
    int32_t *deg = buf<int32_t>(h, h->deg, (size_t)m);
    launch_fill_i32(deg, m, 0, st);
    a.deg = deg;
    tm.mark();
    launch_pair_count(a, st);
    tm.mark();
    int64_t *rowptr = buf<int64_t>(h, h->rowptr, (size_t)m + 1);
    void *tmp = h->arena.ensure(h->scan_tmp, scan_tmp_bytes(std::max<int64_t>(P, m)));
    exclusive_scan_i32_to_i64(deg, rowptr, m, true, tmp, st);
    const int64_t total = read_scalar(h, rowptr + m);
    if (total % 2) throw Error(PICASSO_EINTERNAL, "odd CSR size");
    const int64_t bytes = total * (int64_t)sizeof(int32_t);
    if (h->mem_budget > 0 && bytes > h->mem_budget)
        throw Error(PICASSO_ENOMEM, "conflict graph needs " + std::to_string(bytes) + " bytes, budget " +
                                        std::to_string(h->mem_budget));
    int32_t *adj = buf<int32_t>(h, h->adj, (size_t)std::max<int64_t>(total, 1));
    int32_t *cursor = buf<int32_t>(h, h->cursor32, (size_t)m);
    launch_fill_i32(cursor, m, 0, st);
    a.rowptr = rowptr;
    a.cursor = cursor;
    a.adj = adj;
    tm.mark();
    launch_pair_fill(a, st);
    tm.mark();
    if (ms_count) *ms_count = tm.ms(0, 1);
    if (ms_fill) *ms_fill = tm.ms(2, 3);
    return total / 2;
}

// Jones-Plassmann rounds until every vertex is decided.  Result in h->col.
int32_t color_graph(picasso_ctx *h, int64_t m, int32_t T)
{
    hipStream_t st = h->stream;
    ColorArgs c{};
    c.m = m;
    c.rowptr = static_cast<const int64_t *>(h->rowptr.p);
    c.adj = static_cast<const int32_t *>(h->adj.p);
    c.prio = static_cast<const uint64_t *>(h->prio.p);
    c.lists = static_cast<const uint32_t *>(h->lists.p);
    c.T = T;
    c.col = buf<int32_t>(h, h->col, (size_t)m);
    c.cursor = buf<int64_t>(h, h->cursor64, (size_t)m);
    c.fw = (T + 63) / 64;
    c.forbid = buf<uint64_t>(h, h->forbid, (size_t)m * c.fw);
    unsigned long long *sc = buf<unsigned long long>(h, h->scalars, 8);
    c.progress = sc + 1;
    launch_fill_u32(reinterpret_cast<uint32_t *>(sc + 1), 2, 0u, st);
    launch_color_init(c, st);
    int32_t rounds = 0;
    int batch = 4;
    while (true) {
        for (int r = 0; r < batch; ++r) launch_color_round(c, st);
        rounds += batch;
        const unsigned long long done = read_scalar(h, c.progress);
        if ((int64_t)done >= m) break;
        // every round decides at least the first undecided vertex in the order
        if (rounds > m + 64) throw Error(PICASSO_EINTERNAL, "list colouring made no progress");
        if (batch < 64) batch *= 2;
    }
    return rounds;
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

void init_ids(picasso_ctx *h, int64_t m);

int64_t color_all(picasso_ctx *h, uint64_t seed, double frac, double alpha, int32_t rel, int32_t *d_out)
{
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = h->stream;
    picasso_stats &S = h->stats;
    std::memset(&S, 0, sizeof(S));
    S.n = h->n;
    h->arena.peak = h->arena.live;
    launch_fill_i32(d_out, h->n, -1, st);
    init_ids(h, h->n);
    int64_t m = h->n, offset = 0, n_colors = 0;
    uint32_t ell = 1;
    while (m > 0) {
        int64_t P;
        int32_t T;
        params(m, frac, alpha, h->fixed_T, P, T);
        if (T > PICASSO_MAX_T) throw Error(PICASSO_EINVAL, "list size " + std::to_string(T) + " exceeds PICASSO_MAX_T");
        if (P > INT32_MAX) throw Error(PICASSO_EINVAL, "palette too large");
        picasso_iter_stats it{};
        it.m = m;
        it.P = P;
        it.T = T;
        it.offset = offset;
        it.pair_path = PICASSO_PATH_VALU;
        Timer tm(h);
        tm.mark();
        const int32_t *d_ids = static_cast<const int32_t *>(h->ids.p);
        it.pair_tests = build_lists_and_buckets(h, seed, ell, m, d_ids, P, T);
        tm.mark();
        it.edges = build_conflict_graph(h, m, P, T, rel, &it.ms_count, &it.ms_fill);
        tm.mark();
        it.jp_rounds = color_graph(h, m, T);
        tm.mark();
        // global colours, used-colour count, next vertex set
        uint32_t *used = buf<uint32_t>(h, h->used, (size_t)(P + 31) / 32);
        launch_fill_u32(used, (P + 31) / 32, 0u, st);
        unsigned long long *sc = buf<unsigned long long>(h, h->scalars, 8);
        launch_fill_u32(reinterpret_cast<uint32_t *>(sc + 2), 2, 0u, st);
        int32_t *flags = buf<int32_t>(h, h->flags, (size_t)m);
        launch_finish_iteration(m, static_cast<const int32_t *>(h->col.p), d_ids, offset, d_out, used, sc + 2, flags,
                                st);
        int64_t *pos = buf<int64_t>(h, h->pos, (size_t)m + 1);
        void *tmp = h->arena.ensure(h->scan_tmp, scan_tmp_bytes(std::max<int64_t>(P, m)));
        exclusive_scan_i32_to_i64(flags, pos, m, true, tmp, st);
        int32_t *next = buf<int32_t>(h, h->next_ids, (size_t)m);
        launch_compact_ids(m, d_ids, flags, pos, next, st);
        tm.mark();
        const int64_t m_next = read_scalar(h, pos + m);
        const int64_t used_now = (int64_t)read_scalar(h, sc + 2);
        it.colored = m - m_next;
        it.ms_lists = tm.ms(0, 1);
        it.ms_color = tm.ms(2, 3);
        it.ms_compact = tm.ms(3, 4);
        if (it.colored <= 0) throw Error(PICASSO_EINTERNAL, "iteration coloured no vertex");
        std::swap(h->ids, h->next_ids);
        n_colors += used_now;
        if (S.n_iters < PICASSO_MAX_ITER_STATS) S.iters[S.n_iters] = it;
        S.n_iters++;
        S.palette_total += P;
        S.pair_tests += it.pair_tests;
        S.edges += it.edges;
        if (it.edges > S.max_edges) S.max_edges = it.edges;
        offset += P;
        m = m_next;
        ++ell;
    }
    PCHECK_HIP(hipStreamSynchronize(st));
    S.n_colors = n_colors;
    S.peak_device_bytes = (int64_t)h->arena.peak;
    S.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return n_colors;
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
    if (rel != PICASSO_REL_ANTICOMMUTE && rel != PICASSO_REL_QWC) throw Error(PICASSO_EINVAL, "unknown relation");
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
        const size_t bytes = (size_t)std::max<int64_t>(n, 1) * W * sizeof(uint64_t);
        uint64_t *dx = static_cast<uint64_t *>(h->arena.ensure(h->x, bytes));
        uint64_t *dz = static_cast<uint64_t *>(h->arena.ensure(h->z, bytes));
        const size_t cb = (size_t)n * W * sizeof(uint64_t);
        if (cb) {
            const hipMemcpyKind kind = device_src ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
            PCHECK_HIP(hipMemcpyAsync(dx, x, cb, kind, h->stream));
            PCHECK_HIP(hipMemcpyAsync(dz, z, cb, kind, h->stream));
        }
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

void picasso_destroy(picasso_handle h)
{
    if (!h) return;
    (void)hipSetDevice(h->device);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    DevBuf *all[] = {&h->x,      &h->z,       &h->ids,     &h->next_ids, &h->lists,    &h->prio,     &h->bcnt,
                     &h->bstart, &h->bmem,    &h->bslot,   &h->deg,      &h->rowptr,   &h->adj,      &h->cursor32,
                     &h->col,    &h->cursor64, &h->forbid, &h->flags,    &h->pos,      &h->used,     &h->scan_tmp,
                     &h->scalars, &h->out_colors};
    for (DevBuf *b : all) h->arena.release(*b);
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
            check_color_args(palette_frac, list_size, relation);
            if (h->n > 0 && !out_colors) throw Error(PICASSO_EINVAL, "null output");
            if (h->n == 0) {
                std::memset(&h->stats, 0, sizeof(h->stats));
                return 0;
            }
            return color_all(h, seed, palette_frac, list_size, relation, out_colors);
        },
        PICASSO_EINTERNAL);
}

int64_t picasso_color(picasso_handle h, uint64_t seed, double palette_frac, double list_size, int32_t relation,
                      int32_t *out_colors)
{
    return guarded(
        [&]() -> int64_t {
            check_handle(h);
            check_color_args(palette_frac, list_size, relation);
            if (h->n > 0 && !out_colors) throw Error(PICASSO_EINVAL, "null output");
            if (h->n == 0) {
                std::memset(&h->stats, 0, sizeof(h->stats));
                return 0;
            }
            int32_t *d_out = buf<int32_t>(h, h->out_colors, (size_t)h->n);
            const int64_t nc = color_all(h, seed, palette_frac, list_size, relation, d_out);
            const auto t0 = std::chrono::steady_clock::now();
            download(h, out_colors, d_out, (size_t)h->n * sizeof(int32_t));
            h->stats.ms_total +=
                std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            return nc;
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
            check_subset(h, m, ids, P, T);
            if (m > 0 && !out_lists) throw Error(PICASSO_EINVAL, "null output");
            if (m == 0) return PICASSO_OK;
            int32_t *d_ids = buf<int32_t>(h, h->ids, (size_t)m);
            upload(h, d_ids, ids, (size_t)m * sizeof(int32_t));
            uint32_t *lists = buf<uint32_t>(h, h->lists, (size_t)m * T);
            uint64_t *prio = buf<uint64_t>(h, h->prio, (size_t)m);
            launch_sample_lists(seed, (uint32_t)ell, m, d_ids, P, T, lists, prio, h->stream);
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
            check_subset(h, m, ids, P, T);
            check_rel(relation);
            if (m == 0) {
                if (out_rowptr) out_rowptr[0] = 0;
                return 0;
            }
            int32_t *d_ids = buf<int32_t>(h, h->ids, (size_t)m);
            upload(h, d_ids, ids, (size_t)m * sizeof(int32_t));
            build_lists_and_buckets(h, seed, (uint32_t)ell, m, d_ids, P, T);
            const int64_t edges = build_conflict_graph(h, m, P, T, relation, nullptr, nullptr);
            if (out_rowptr) download(h, out_rowptr, h->rowptr.p, (size_t)(m + 1) * sizeof(int64_t));
            if (out_adj && 2 * edges <= adj_cap) download(h, out_adj, h->adj.p, (size_t)(2 * edges) * sizeof(int32_t));
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
            upload(h, buf<uint64_t>(h, h->prio, (size_t)m), prio, (size_t)m * sizeof(uint64_t));
            upload(h, buf<uint32_t>(h, h->lists, (size_t)m * T), lists, (size_t)m * T * sizeof(uint32_t));
            upload(h, buf<int64_t>(h, h->rowptr, (size_t)m + 1), rowptr, (size_t)(m + 1) * sizeof(int64_t));
            upload(h, buf<int32_t>(h, h->adj, (size_t)std::max<int64_t>(total, 1)), adj,
                   (size_t)total * sizeof(int32_t));
            color_graph(h, m, T);
            download(h, out_col, h->col.p, (size_t)m * sizeof(int32_t));
            int64_t colored = 0;
            for (int64_t i = 0; i < m; ++i) colored += out_col[i] >= 0;
            return colored;
        },
        PICASSO_EINTERNAL);
}

}  // extern "C"
