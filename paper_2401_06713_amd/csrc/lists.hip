// Random colour lists (Alg. 1 assign_rand_list_colors) and colour buckets.
//
// Lists: each vertex gets a uniform T-subset of the palette [0, P) (Sec. IV:
// colours drawn uniformly at random), drawn with Floyd's algorithm, one
// Philox4x32-10 value per step keyed by (seed; original vertex id, step,
// iteration), kept sorted in LDS while it is built.  Keys use the original
// id, so a list does not depend on where the vertex sits in the compacted
// vertex set or on the thread that draws it.
//
// Buckets: B_c = {(vertex, slot) : L(vertex)[slot] = c}, built by a count
// (one atomic per list entry), an exclusive scan and a scatter.  Only
// vertices inside one bucket can conflict through colour c, so the pair
// kernels test pairs inside buckets instead of all C(m,2) pairs.
#include "common.h"

namespace picasso {
namespace {

// Instance of active vertex v: the last record with vstart <= v.
__device__ __forceinline__ int32_t find_instance_of_vertex(const Batch &b, int64_t v)
{
    int32_t lo = 0, hi = b.nb;  // inst[lo].vstart <= v < inst[hi].vstart
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (b.inst[mid].vstart <= v) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ void vertex_table_kernel(Batch b, int64_t m, int32_t *__restrict__ vinst, int64_t *__restrict__ loff)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v <= m; v += (int64_t)gridDim.x * blockDim.x) {
        if (v == m) {
            const InstRec &r = b.inst[b.nb - 1];
            loff[m] = r.loff + r.m * r.T;
        } else {
            const int32_t i = find_instance_of_vertex(b, v);
            const InstRec &r = b.inst[i];
            vinst[v] = i;
            loff[v] = r.loff + (v - r.vstart) * r.T;
        }
    }
}

__global__ void bucket_table_kernel(Batch b, int64_t P, int32_t *__restrict__ binst)
{
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < P; c += (int64_t)gridDim.x * blockDim.x) {
        int32_t lo = 0, hi = b.nb;  // inst[lo].pal <= c < inst[hi].pal
        while (hi - lo > 1) {
            const int32_t mid = (lo + hi) >> 1;
            if (b.inst[mid].pal <= c) lo = mid;
            else hi = mid;
        }
        binst[c] = lo;
    }
}

// One thread per vertex.  s[T_max][blockDim] holds each thread's sorted set
// (slot-major, so consecutive threads hit consecutive LDS banks).  The draws
// use the instance's seed and palette and the vertex's id within its
// instance; the stored colour is shifted by the instance's palette start.
__global__ void sample_lists_kernel(Batch b, uint32_t ell, int64_t m, const int32_t *__restrict__ ids,
                                    uint32_t *__restrict__ lists, uint64_t *__restrict__ prio)
{
    extern __shared__ uint32_t s[];
    __shared__ int uniform;
    const int B = blockDim.x, t = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * B;
    const int64_t i = r0 + t;
    const int64_t rows = (m - r0) < B ? (m - r0) : B;
    if (t == 0) uniform = b.vinst[r0] == b.vinst[r0 + rows - 1];
    int32_t T = 0;
    uint32_t pal = 0;
    if (i < m) {
        const InstRec &r = b.inst[b.vinst[i]];
        T = r.T;
        pal = (uint32_t)r.pal;
        const int64_t P = r.P;
        const uint32_t v = (uint32_t)(ids[i] - r.sbase);
        int cnt = 0;
        for (int step = 0; step < T; ++step) {
            const uint64_t j = (uint64_t)(P - T + step);
            const uint64_t rnd = philox_draw(r.seed, v, (uint32_t)step, ell, TAG_LIST);
            const uint32_t cand = (uint32_t)__umul64hi(rnd, j + 1);  // in [0, j]
            // binary search for cand among s[0..cnt)
            int lo = 0, hi = cnt;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (s[mid * B + t] < cand) lo = mid + 1;
                else hi = mid;
            }
            if (lo < cnt && s[lo * B + t] == cand) {
                // present: take j, larger than every value drawn so far
                s[cnt * B + t] = (uint32_t)j;
            } else {
                for (int k = cnt; k > lo; --k) s[k * B + t] = s[(k - 1) * B + t];
                s[lo * B + t] = cand;
            }
            ++cnt;
        }
        if (prio) prio[i] = philox_draw(r.seed, v, 0, ell, TAG_PRIO);
    }
    __syncthreads();
    if (uniform) {
        // one instance: the block's rows are one run of lists, written coalesced
        const InstRec &r = b.inst[b.vinst[r0]];
        const int32_t Tu = r.T;
        const uint32_t pu = (uint32_t)r.pal;
        const int64_t words = rows * Tu;
        uint32_t *dst = lists + b.loff[r0];
        for (int64_t e = t; e < words; e += B) {
            const int64_t row = e / Tu, slot = e - row * Tu;
            dst[e] = pu + s[slot * B + row];
        }
    } else if (i < m) {
        uint32_t *dst = lists + b.loff[i];
        for (int k = 0; k < T; ++k) dst[k] = pal + s[k * B + t];
    }
}

__global__ void bucket_count_kernel(const uint32_t *__restrict__ lists, int64_t entries, uint32_t *__restrict__ bcnt)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < entries; e += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&bcnt[lists[e]], 1u);
}

__global__ void bucket_scatter_kernel(const uint32_t *__restrict__ lists, int64_t m, const int64_t *__restrict__ loff,
                                      const int64_t *__restrict__ bstart, uint32_t *__restrict__ bfill,
                                      uint32_t *__restrict__ bmem, slot_t *__restrict__ bslot)
{
    // The position in the bucket comes back from an atomic add; eight of
    // them are issued before the first result is used, so a thread waits
    // for one atomic round trip per eight list entries, not per entry.
    // (The order within a bucket is arbitrary: the sort that follows orders
    // the members by their unique (priority, id) keys.)
    constexpr int kGroup = 8;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < m; v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e0 = loff[v], T = loff[v + 1] - e0;
        for (int64_t k0 = 0; k0 < T; k0 += kGroup) {
            uint32_t c[kGroup], pos[kGroup];
            int64_t base[kGroup];
#pragma unroll
            for (int j = 0; j < kGroup; ++j)
                if (k0 + j < T) c[j] = lists[e0 + k0 + j];
#pragma unroll
            for (int j = 0; j < kGroup; ++j)
                if (k0 + j < T) {
                    base[j] = bstart[c[j]];
                    pos[j] = atomicAdd(&bfill[c[j]], 1u);
                }
#pragma unroll
            for (int j = 0; j < kGroup; ++j)
                if (k0 + j < T) {
                    const int64_t at = base[j] + pos[j];
                    bmem[at] = (uint32_t)v;
                    bslot[at] = (slot_t)(k0 + j);
                }
        }
    }
}

__global__ void check_padding_kernel(const uint64_t *x, const uint64_t *z, int64_t n, int32_t q, int32_t *bad)
{
    const int W = (q + 63) / 64, rem = q % 64;
    if (rem == 0) return;
    const uint64_t mask = ~((1ull << rem) - 1ull);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if ((x[i * W + W - 1] | z[i * W + W - 1]) & mask) atomicExch(bad, 1);
}

__global__ void bucket_pairs_kernel(const uint32_t *__restrict__ bcnt, int64_t P, unsigned long long *pairs)
{
    unsigned long long s = 0, mx = 0;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < P; c += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long k = bcnt[c];
        s += k * (k - (k > 0)) / 2;
        mx = k > mx ? k : mx;
    }
    for (int d = 32; d > 0; d >>= 1) {
        s += __shfl_down(s, d, 64);
        const unsigned long long o = __shfl_down(mx, d, 64);
        mx = o > mx ? o : mx;
    }
    // one pair of atomics per workgroup: they all land on one line
    __shared__ unsigned long long ws[4], wm[4];
    if ((threadIdx.x & 63) == 0) {
        ws[threadIdx.x >> 6] = s;
        wm[threadIdx.x >> 6] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
            s += ws[w];
            mx = wm[w] > mx ? wm[w] : mx;
        }
        if (s) atomicAdd(&pairs[0], s);
        atomicMax(&pairs[1], mx);
    }
}

// ---- bucket order ----------------------------------------------------------
// Members of a bucket sorted by (priority, local index): the order in which
// the sequential colouring visits them.  Buckets up to kSortCap members are
// sorted in LDS by a bitonic network; larger ones rank each member by
// counting the members before it.
constexpr int kSortThreads = 256;
constexpr int kSortCap = 2048;

__device__ __forceinline__ bool key_less(uint64_t pa, uint32_t va, uint64_t pb, uint32_t vb)
{
    return pa < pb || (pa == pb && va < vb);
}

__global__ void __launch_bounds__(kSortThreads) bucket_sort_kernel(const int64_t *__restrict__ bstart, int64_t P,
                                                                   uint32_t *__restrict__ bmem,
                                                                   slot_t *__restrict__ bslot,
                                                                   const uint64_t *__restrict__ prio,
                                                                   int64_t *__restrict__ pos_of,
                                                                   int64_t *__restrict__ bent,
                                                                   const int64_t *__restrict__ loff)
{
    __shared__ uint64_t key[kSortCap];
    __shared__ uint32_t vid[kSortCap];
    __shared__ slot_t sl[kSortCap];
    const int t = threadIdx.x;
    for (int64_t c = blockIdx.x; c < P; c += gridDim.x) {
        const int64_t base = bstart[c];
        const int64_t S = bstart[c + 1] - base;
        if (S > kSortCap) continue;
        if (S == 1 && t == 0) {
            const int64_t en = loff[bmem[base]] + bslot[base];
            pos_of[en] = base;
            bent[base] = en;
        }
        if (S < 2) continue;
        int N = 2;
        while (N < S) N <<= 1;
        __syncthreads();
        for (int e = t; e < N; e += kSortThreads) {
            if (e < S) {
                const uint32_t v = bmem[base + e];
                key[e] = prio[v];
                vid[e] = v;
                sl[e] = bslot[base + e];
            } else {
                key[e] = ~0ull;
                vid[e] = 0xFFFFFFFFu;
                sl[e] = 0;
            }
        }
        __syncthreads();
        for (int k = 2; k <= N; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int e = t; e < N; e += kSortThreads) {
                    const int f = e ^ j;
                    if (f > e) {
                        const bool up = (e & k) == 0;
                        const bool gt = key_less(key[f], vid[f], key[e], vid[e]);
                        if (gt == up) {
                            const uint64_t tk = key[e];
                            key[e] = key[f];
                            key[f] = tk;
                            const uint32_t tv = vid[e];
                            vid[e] = vid[f];
                            vid[f] = tv;
                            const slot_t ts = sl[e];
                            sl[e] = sl[f];
                            sl[f] = ts;
                        }
                    }
                }
                __syncthreads();
            }
        }
        for (int e = t; e < S; e += kSortThreads) {
            bmem[base + e] = vid[e];
            bslot[base + e] = sl[e];
            const int64_t en = loff[vid[e]] + sl[e];
            pos_of[en] = base + e;
            bent[base + e] = en;
        }
    }
}

// Buckets above kSortCap: each member's rank is the number of members with a
// smaller (priority, vertex) key.  The bucket's keys are compared in tiles
// staged in LDS (one gather of the priorities per tile); each pass ranks
// kSortThreads members, one per thread.
constexpr int kRankTile = 2048;

__global__ void __launch_bounds__(kSortThreads) bucket_rank_kernel(const int64_t *__restrict__ bstart, int64_t P,
                                                                   const uint32_t *__restrict__ bmem,
                                                                   const slot_t *__restrict__ bslot,
                                                                   const uint64_t *__restrict__ prio,
                                                                   uint32_t *__restrict__ out_mem,
                                                                   slot_t *__restrict__ out_slot)
{
    __shared__ uint64_t tkey[kRankTile];
    __shared__ uint32_t tvid[kRankTile];
    for (int64_t c = blockIdx.x; c < P; c += gridDim.x) {
        const int64_t base = bstart[c];
        const int64_t S = bstart[c + 1] - base;
        if (S <= kSortCap) continue;
        for (int64_t p0 = 0; p0 < S; p0 += kSortThreads) {
            const int64_t p = p0 + threadIdx.x;
            uint32_t vp = 0;
            uint64_t kp = 0;
            if (p < S) {
                vp = bmem[base + p];
                kp = prio[vp];
            }
            int64_t rank = 0;
            for (int64_t t0 = 0; t0 < S; t0 += kRankTile) {
                const int64_t nt = S - t0 < kRankTile ? S - t0 : kRankTile;
                __syncthreads();
                for (int64_t i = threadIdx.x; i < nt; i += kSortThreads) {
                    const uint32_t v = bmem[base + t0 + i];
                    tvid[i] = v;
                    tkey[i] = prio[v];
                }
                __syncthreads();
                if (p < S)
                    for (int64_t i = 0; i < nt; ++i) rank += key_less(tkey[i], tvid[i], kp, vp);
            }
            if (p < S) {
                out_mem[base + rank] = vp;
                out_slot[base + rank] = bslot[base + p];
            }
        }
    }
}

__global__ void __launch_bounds__(kSortThreads) bucket_rank_copy_kernel(const int64_t *__restrict__ bstart, int64_t P,
                                                                        uint32_t *__restrict__ bmem,
                                                                        slot_t *__restrict__ bslot,
                                                                        const uint32_t *__restrict__ tmp_mem,
                                                                        const slot_t *__restrict__ tmp_slot,
                                                                        int64_t *__restrict__ pos_of,
                                                                        int64_t *__restrict__ bent,
                                                                        const int64_t *__restrict__ loff)
{
    for (int64_t c = blockIdx.x; c < P; c += gridDim.x) {
        const int64_t base = bstart[c];
        const int64_t S = bstart[c + 1] - base;
        if (S <= kSortCap) continue;
        for (int64_t p = threadIdx.x; p < S; p += blockDim.x) {
            const uint32_t v = tmp_mem[base + p];
            const slot_t k = tmp_slot[base + p];
            bmem[base + p] = v;
            bslot[base + p] = k;
            const int64_t en = loff[v] + k;
            pos_of[en] = base + p;
            bent[base + p] = en;
        }
    }
}

__global__ void bucket_shapes_kernel(const int64_t *__restrict__ bstart, int64_t P, int64_t *__restrict__ tiles,
                                     int64_t *__restrict__ words)
{
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < P; c += (int64_t)gridDim.x * blockDim.x) {
        const int64_t S = bstart[c + 1] - bstart[c];
        const int64_t nw = (S + 63) >> 6;
        tiles[c] = nw;
        words[c] = S * nw;
    }
}

template <typename V>
__global__ void fill_kernel(V *p, int64_t n, V v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

unsigned grid_for(int64_t work, int threads, unsigned cap = 65535u * 4)
{
    int64_t b = (work + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

}  // namespace

void launch_vertex_table(const Batch &b, int64_t m, int32_t *vinst, int64_t *loff, hipStream_t st)
{
    if (b.nb <= 0) throw Error(PICASSO_EINTERNAL, "vertex table of an empty batch");
    vertex_table_kernel<<<grid_for(m + 1, 256), 256, 0, st>>>(b, m, vinst, loff);
    PCHECK_LAUNCH();
}

void launch_bucket_table(const Batch &b, int64_t P, int32_t *binst, hipStream_t st)
{
    if (P <= 0) return;
    bucket_table_kernel<<<grid_for(P, 256), 256, 0, st>>>(b, P, binst);
    PCHECK_LAUNCH();
}

void launch_sample_lists(const Batch &b, uint32_t ell, int64_t m, const int32_t *ids, int32_t T_max,
                         uint32_t *lists, uint64_t *prio, hipStream_t st)
{
    if (m <= 0) return;
    // lists are built in LDS, T_max x B words: at most 64 KB
    const int B = T_max <= 64 ? 256 : T_max <= 128 ? 128 : T_max <= 256 ? 64 : T_max <= 512 ? 32 : 16;
    if (T_max > PICASSO_MAX_T) throw Error(PICASSO_EINVAL, "list size above PICASSO_MAX_T");
    const size_t lds = (size_t)T_max * B * sizeof(uint32_t);
    const int64_t blocks = (m + B - 1) / B;
    sample_lists_kernel<<<(unsigned)blocks, B, lds, st>>>(b, ell, m, ids, lists, prio);
    PCHECK_LAUNCH();
}

void launch_bucket_count(const uint32_t *lists, int64_t entries, uint32_t *bcnt, hipStream_t st)
{
    if (entries <= 0) return;
    bucket_count_kernel<<<grid_for(entries, 256), 256, 0, st>>>(lists, entries, bcnt);
    PCHECK_LAUNCH();
}

void launch_bucket_scatter(const uint32_t *lists, int64_t m, const int64_t *loff, const int64_t *bstart,
                           uint32_t *bfill, uint32_t *bmem, slot_t *bslot, hipStream_t st)
{
    if (m <= 0) return;
    bucket_scatter_kernel<<<grid_for(m, 256), 256, 0, st>>>(lists, m, loff, bstart, bfill, bmem, bslot);
    PCHECK_LAUNCH();
}

void launch_check_padding(const uint64_t *x, const uint64_t *z, int64_t n, int32_t q, int32_t *bad, hipStream_t st)
{
    if (n <= 0) return;
    check_padding_kernel<<<grid_for(n, 256), 256, 0, st>>>(x, z, n, q, bad);
    PCHECK_LAUNCH();
}

void launch_bucket_pairs(const uint32_t *bcnt, int64_t P, unsigned long long *pairs, hipStream_t st)
{
    if (P <= 0) return;
    bucket_pairs_kernel<<<grid_for(P, 256, 128), 256, 0, st>>>(bcnt, P, pairs);
    PCHECK_LAUNCH();
}

void launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t st)
{
    if (n <= 0) return;
    fill_kernel<int32_t><<<grid_for(n, 256), 256, 0, st>>>(p, n, v);
    PCHECK_LAUNCH();
}

void launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t st)
{
    if (n <= 0) return;
    fill_kernel<uint32_t><<<grid_for(n, 256), 256, 0, st>>>(p, n, v);
    PCHECK_LAUNCH();
}

void launch_fill_u64(uint64_t *p, int64_t n, uint64_t v, hipStream_t st)
{
    if (n <= 0) return;
    fill_kernel<uint64_t><<<grid_for(n, 256), 256, 0, st>>>(p, n, v);
    PCHECK_LAUNCH();
}

void launch_fill_u8(uint8_t *p, int64_t n, uint8_t v, hipStream_t st)
{
    if (n <= 0) return;
    fill_kernel<uint8_t><<<grid_for(n, 256), 256, 0, st>>>(p, n, v);
    PCHECK_LAUNCH();
}

void launch_bucket_sort(const int64_t *bstart, int64_t P, uint32_t *bmem, slot_t *bslot, const uint64_t *prio,
                        int64_t *pos_of, int64_t *bent, const int64_t *loff, bool has_large, uint32_t *tmp_mem,
                        slot_t *tmp_slot, hipStream_t st)
{
    if (P <= 0) return;
    const unsigned grid = (unsigned)(P < (1 << 20) ? P : (1 << 20));
    bucket_sort_kernel<<<grid, kSortThreads, 0, st>>>(bstart, P, bmem, bslot, prio, pos_of, bent, loff);
    PCHECK_LAUNCH();
    if (has_large) {
        bucket_rank_kernel<<<grid, kSortThreads, 0, st>>>(bstart, P, bmem, bslot, prio, tmp_mem, tmp_slot);
        PCHECK_LAUNCH();
        bucket_rank_copy_kernel<<<grid, kSortThreads, 0, st>>>(bstart, P, bmem, bslot, tmp_mem, tmp_slot, pos_of,
                                                                 bent, loff);
        PCHECK_LAUNCH();
    }
}

void launch_bucket_shapes(const int64_t *bstart, int64_t P, int64_t *tiles, int64_t *words, hipStream_t st)
{
    if (P <= 0) return;
    bucket_shapes_kernel<<<grid_for(P, 256), 256, 0, st>>>(bstart, P, tiles, words);
    PCHECK_LAUNCH();
}

}  // namespace picasso
