// Stable least-significant-digit radix sort of (key, value) pairs, and the
// colour-bucket build that uses it.
//
// Each pass sorts by one 8- or 9-bit digit: a digit histogram per tile of
// kTile elements, an exclusive scan over (digit, tile) -- digit-major, so a
// tile's elements of digit d land after every earlier tile's -- and a
// stable scatter.  Within a tile, elements are ranked in input order: per
// round of 256 elements, each wave finds the lanes with its digit by one
// ballot per digit bit, and per-wave digit counts in LDS order the four
// waves.  The ranked tile is staged in LDS in digit order and written out
// from there, in runs of one digit.  Tiles go to the XCDs in contiguous
// runs: a digit's runs from neighbouring tiles are neighbours in the output,
// as are the tiles' entries in the (digit, tile) count and offset tables, so
// their partly written or read cache lines meet in one L2.
//
// Bucket build (Alg. 1 buckets of list entries, members in the colouring
// order): the vertices are sorted by (priority, index) (four passes over the
// priority's high half, stable from ascending index, then the rare runs of
// equal high halves ordered by the whole priority), their list entries are
// emitted in that order, and a stable sort by colour then leaves every
// bucket's members in priority order -- count, scatter and the per-bucket
// sort in one pass over the entries per colour digit, with no atomics on
// global counters.
#include <algorithm>

#include "common.h"

namespace picasso {
namespace {

constexpr int kRThreads = 256;
constexpr int kRItems = 8;
constexpr int64_t kRTile = (int64_t)kRThreads * kRItems;
constexpr int kMaxDigitBits = 9;

template <typename K, int DB>
__device__ __forceinline__ uint32_t digit_of(K key, int shift)
{
    return (uint32_t)(key >> shift) & ((1u << DB) - 1u);
}

template <typename K, int DB>
__global__ void __launch_bounds__(kRThreads) radix_hist_kernel(const K *__restrict__ keys, int64_t n, int shift,
                                                               int64_t ntiles, uint32_t *__restrict__ counts)
{
    constexpr int kBins = 1 << DB;
    __shared__ uint32_t h[kBins];
    for (int d = threadIdx.x; d < kBins; d += kRThreads) h[d] = 0u;
    __syncthreads();
    const int64_t tile = xcd_item(blockIdx.x, ntiles);
    const int64_t base = tile * kRTile;
#pragma unroll
    for (int i = 0; i < kRItems; ++i) {
        const int64_t g = base + (int64_t)i * kRThreads + threadIdx.x;
        if (g < n) atomicAdd(&h[digit_of<K, DB>(keys[g], shift)], 1u);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < kBins; d += kRThreads) counts[(int64_t)d * ntiles + tile] = h[d];
}

// Scatter of one tile: each element's rank among the tile's elements of its
// digit (stable, in input order) places it in LDS in digit order; the tile is
// then written out from LDS, so consecutive threads write consecutive
// positions of one digit's run instead of one scattered element each.
template <typename K, int DB>
__global__ void __launch_bounds__(kRThreads) radix_scatter_kernel(const K *__restrict__ keys,
                                                                  const uint32_t *__restrict__ vals, int64_t n,
                                                                  int shift, int64_t ntiles,
                                                                  const uint32_t *__restrict__ counts,
                                                                  const int64_t *__restrict__ offsets,
                                                                  K *__restrict__ out_keys,
                                                                  uint32_t *__restrict__ out_vals)
{
    constexpr int kBins = 1 << DB;
    constexpr int kPer = kBins / kRThreads;  // bins per thread in the scan (1 or 2)
    __shared__ int64_t off[kBins];          // global start of each digit's run of this tile
    __shared__ uint32_t lstart[kBins];      // start of each digit in the tile (exclusive scan of its counts)
    __shared__ uint32_t running[kBins];
    __shared__ uint32_t wcnt[kRThreads / 64][kBins];
    __shared__ uint32_t wtot[kRThreads / 64];
    __shared__ K skey[kRTile];
    __shared__ uint32_t sval[kRTile];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t tile = xcd_item(blockIdx.x, ntiles);
    // the tile's digit counts, scanned: kPer bins per thread, then the waves
    uint32_t cnt[kPer], sum = 0u;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int d = t * kPer + j;
        off[d] = offsets[(int64_t)d * ntiles + tile];
        running[d] = 0u;
        cnt[j] = counts[(int64_t)d * ntiles + tile];
        sum += cnt[j];
    }
    uint32_t inc = sum;
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = __shfl_up(inc, d, 64);
        if (lane >= d) inc += o;
    }
    if (lane == 63) wtot[wave] = inc;
    __syncthreads();
    uint32_t before = inc - sum;
    for (int w = 0; w < wave; ++w) before += wtot[w];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        lstart[t * kPer + j] = before;
        before += cnt[j];
    }
    const uint64_t lanes_below = (1ull << lane) - 1ull;
    const int64_t base = tile * kRTile;
    for (int i = 0; i < kRItems; ++i) {
        for (int w = 0; w < kRThreads / 64; ++w)
            for (int d = t; d < kBins; d += kRThreads) wcnt[w][d] = 0u;
        __syncthreads();
        const int64_t g = base + (int64_t)i * kRThreads + t;
        const bool valid = g < n;
        K key = 0;
        uint32_t val = 0, d = 0;
        if (valid) {
            key = keys[g];
            val = vals[g];
            d = digit_of<K, DB>(key, shift);
        }
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < DB; ++b) {
            const uint64_t bal = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? bal : ~bal;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lanes_below);
        const bool leader = valid && (peers >> lane) == 1ull;  // highest lane of its digit
        if (leader) wcnt[wave][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t r = running[d];
            for (int w = 0; w < wave; ++w) r += wcnt[w][d];
            const uint32_t li = lstart[d] + r + rank;
            if (li < (uint32_t)kRTile) {
                skey[li] = key;
                sval[li] = val;
            }
        }
        __syncthreads();
        for (int dd = t; dd < kBins; dd += kRThreads) {
            uint32_t add = 0u;
            for (int w = 0; w < kRThreads / 64; ++w) add += wcnt[w][dd];
            running[dd] += add;
        }
        __syncthreads();
    }
    // out of LDS in digit order
    const int64_t m = n - base < kRTile ? n - base : kRTile;
    for (int j = t; j < m; j += kRThreads) {
        const K key = skey[j];
        const uint32_t d = digit_of<K, DB>(key, shift);
        const int64_t pos = off[d] + (j - (int64_t)lstart[d]);
        if (pos >= 0 && pos < n) {
            out_keys[pos] = key;
            out_vals[pos] = sval[j];
        }
    }
}

// ---- bucket build ------------------------------------------------------------

// Sort keys of the vertex order: the high half of each 64-bit priority,
// with the vertex index as the value.
__global__ void prio_keys_kernel(const uint64_t *__restrict__ prio, int64_t m, uint32_t *__restrict__ hi,
                                 uint32_t *__restrict__ idx)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        hi[i] = (uint32_t)(prio[i] >> 32);
        idx[i] = (uint32_t)i;
    }
}

// After the stable sort by the high halves, every run of equal high halves
// is in index order; the thread at the start of a run puts it in (priority,
// index) order by insertion on the full priorities.  Runs are short: of m
// random priorities, about m^2 / 2^33 pairs share a high half.
__global__ void prio_ties_kernel(const uint32_t *__restrict__ hi, uint32_t *__restrict__ perm,
                                 const uint64_t *__restrict__ prio, int64_t m)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t h = hi[i];
        if (i + 1 >= m || hi[i + 1] != h) continue;
        if (i > 0 && hi[i - 1] == h) continue;
        int64_t end = i + 2;
        while (end < m && hi[end] == h) ++end;
        for (int64_t j = i + 1; j < end; ++j) {
            const uint32_t v = perm[j];
            const uint64_t pv = prio[v];
            int64_t k = j;
            while (k > i) {
                const uint32_t u = perm[k - 1];
                const uint64_t pu = prio[u];
                if (pu < pv || (pu == pv && u < v)) break;
                perm[k] = u;
                --k;
            }
            perm[k] = v;
        }
    }
}

// List sizes in priority order (vertex perm[r] at rank r).
__global__ void ranked_sizes_kernel(const uint32_t *__restrict__ perm, int64_t m, const int64_t *__restrict__ loff,
                                    int32_t *__restrict__ tr)
{
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m; r += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t v = perm[r];
        tr[r] = (int32_t)(loff[v + 1] - loff[v]);
    }
}

// The list entries of the vertices in priority order: (colour, entry index).
// A workgroup takes kEmitRanks consecutive ranks and strides over their
// output range, so that consecutive threads write consecutive entries (and
// read consecutive entries of one list); each thread finds its rank by a
// binary search of the ranks' output offsets, kept in LDS.
constexpr int kEmitRanks = 256;

__global__ void __launch_bounds__(256) emit_ranked_kernel(const uint32_t *__restrict__ perm, int64_t m,
                                                          const int64_t *__restrict__ loff,
                                                          const int64_t *__restrict__ at,
                                                          const uint32_t *__restrict__ lists,
                                                          uint32_t *__restrict__ keys, uint32_t *__restrict__ vals,
                                                          int64_t E)
{
    __shared__ int64_t o[kEmitRanks + 1];  // output offsets of the ranks, and the end
    __shared__ int64_t l[kEmitRanks];      // their first list entries
    for (int64_t r0 = (int64_t)blockIdx.x * kEmitRanks; r0 < m; r0 += (int64_t)gridDim.x * kEmitRanks) {
        const int nr = (int)min<int64_t>(kEmitRanks, m - r0);
        __syncthreads();
        for (int i = threadIdx.x; i <= nr; i += blockDim.x) {
            o[i] = at[r0 + i];  // at holds m + 1 offsets
            if (i < nr) l[i] = loff[perm[r0 + i]];
        }
        __syncthreads();
        const int64_t end = min<int64_t>(o[nr], E);
        for (int64_t x = o[0] + threadIdx.x; x < end; x += blockDim.x) {
            int lo = 0, hi = nr;  // o[lo] <= x < o[hi]
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (o[mid] <= x) lo = mid;
                else hi = mid;
            }
            const int64_t e = l[lo] + (x - o[lo]);
            keys[x] = lists[e];
            vals[x] = (uint32_t)e;
        }
    }
}

// Bucket starts from the colour-sorted keys: position i starts every colour
// in (key[i-1], key[i]]; the end closes the remaining colours.
__global__ void bucket_starts_kernel(const uint32_t *__restrict__ keys, int64_t E, int64_t P,
                                     int64_t *__restrict__ bstart)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= E; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t lo = i == 0 ? 0 : (int64_t)keys[i - 1] + 1;
        const int64_t hi = i == E ? P : (int64_t)keys[i];
        for (int64_t c = lo; c <= hi && c <= P; ++c) bstart[c] = i;
    }
}

__global__ void bucket_counts_kernel(const int64_t *__restrict__ bstart, int64_t P, uint32_t *__restrict__ bcnt)
{
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < P; c += (int64_t)gridDim.x * blockDim.x)
        bcnt[c] = (uint32_t)(bstart[c + 1] - bstart[c]);
}

// Members from the sorted entry indices: the instance by a search of the
// table's list-entry starts, then vertex and slot.
__global__ void bucket_members_kernel(Batch b, const uint32_t *__restrict__ ents, int64_t E,
                                      uint32_t *__restrict__ bmem, slot_t *__restrict__ bslot,
                                      int64_t *__restrict__ pos_of, int64_t *__restrict__ bent)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < E; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = ents[i];
        int32_t lo = 0, hi = b.nb;  // inst[lo].loff <= e < inst[hi].loff
        while (hi - lo > 1) {
            const int32_t mid = (lo + hi) >> 1;
            if (b.inst[mid].loff <= e) lo = mid;
            else hi = mid;
        }
        const InstRec &r = b.inst[lo];
        const int64_t rel = e - r.loff;
        const int64_t v = r.vstart + rel / r.T;
        bmem[i] = (uint32_t)v;
        bslot[i] = (slot_t)(rel % r.T);
        bent[i] = e;
        pos_of[e] = i;
    }
}

unsigned grid_for(int64_t work, int threads, int64_t cap = 65535 * 16)
{
    int64_t b = (work + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

}  // namespace

size_t radix_tmp_bytes(int64_t n)
{
    const int64_t ntiles = std::max<int64_t>((n + kRTile - 1) / kRTile, 1);
    const int64_t nc = ntiles << kMaxDigitBits;
    return (size_t)nc * sizeof(uint32_t) + (size_t)(nc + 1) * sizeof(int64_t) + scan_tmp_bytes(nc + 1) + 512;
}

template <typename K, int DB>
void radix_pass(const K *src_k, const uint32_t *src_v, K *dst_k, uint32_t *dst_v, int64_t n, int shift, int64_t ntiles,
                uint32_t *counts, int64_t *offsets, void *scan_tmp, hipStream_t st)
{
    const int64_t nc = ntiles << DB;
    radix_hist_kernel<K, DB><<<(unsigned)ntiles, kRThreads, 0, st>>>(src_k, n, shift, ntiles, counts);
    PCHECK_LAUNCH();
    exclusive_scan_u32_to_i64(counts, offsets, nc, false, scan_tmp, st);
    radix_scatter_kernel<K, DB><<<(unsigned)ntiles, kRThreads, 0, st>>>(src_k, src_v, n, shift, ntiles, counts,
                                                                        offsets, dst_k, dst_v);
    PCHECK_LAUNCH();
}

// Passes of 9-bit digits where they save a pass over 8-bit ones (18 bits:
// two passes instead of three), else of 8-bit digits.
template <typename K>
int radix_sort_pairs(K *keys, uint32_t *vals, K *keys_alt, uint32_t *vals_alt, int64_t n, int bit_lo, int bit_hi,
                     void *tmp, hipStream_t st)
{
    if (n <= 0) return 0;
    const int64_t ntiles = (n + kRTile - 1) / kRTile;
    if (ntiles > 0x7FFFFFFF) throw Error(PICASSO_EINTERNAL, "radix sort: too many elements");
    const int bits = bit_hi - bit_lo;
    const int p8 = (bits + 7) / 8, p9 = (bits + 8) / 9;
    const int db = p9 < p8 ? 9 : 8;
    const int64_t nc = ntiles << kMaxDigitBits;
    uint32_t *counts = static_cast<uint32_t *>(tmp);
    int64_t *offsets = reinterpret_cast<int64_t *>(
        (reinterpret_cast<uintptr_t>(counts + nc) + 255) & ~(uintptr_t)255);
    void *scan_tmp = reinterpret_cast<void *>((reinterpret_cast<uintptr_t>(offsets + nc + 1) + 255) & ~(uintptr_t)255);
    K *src_k = keys, *dst_k = keys_alt;
    uint32_t *src_v = vals, *dst_v = vals_alt;
    int flips = 0;
    for (int shift = bit_lo; shift < bit_hi; shift += db) {
        if (db == 9)
            radix_pass<K, 9>(src_k, src_v, dst_k, dst_v, n, shift, ntiles, counts, offsets, scan_tmp, st);
        else
            radix_pass<K, 8>(src_k, src_v, dst_k, dst_v, n, shift, ntiles, counts, offsets, scan_tmp, st);
        std::swap(src_k, dst_k);
        std::swap(src_v, dst_v);
        flips ^= 1;
    }
    return flips;
}

template int radix_sort_pairs<uint32_t>(uint32_t *, uint32_t *, uint32_t *, uint32_t *, int64_t, int, int, void *,
                                        hipStream_t);

void launch_prio_keys(const uint64_t *prio, int64_t m, uint32_t *hi, uint32_t *idx, hipStream_t st)
{
    if (m <= 0) return;
    prio_keys_kernel<<<grid_for(m, 256), 256, 0, st>>>(prio, m, hi, idx);
    PCHECK_LAUNCH();
}

void launch_prio_ties(const uint32_t *hi, uint32_t *perm, const uint64_t *prio, int64_t m, hipStream_t st)
{
    if (m <= 1) return;
    prio_ties_kernel<<<grid_for(m, 256), 256, 0, st>>>(hi, perm, prio, m);
    PCHECK_LAUNCH();
}

void launch_ranked_sizes(const uint32_t *perm, int64_t m, const int64_t *loff, int32_t *tr, hipStream_t st)
{
    if (m <= 0) return;
    ranked_sizes_kernel<<<grid_for(m, 256), 256, 0, st>>>(perm, m, loff, tr);
    PCHECK_LAUNCH();
}

void launch_emit_ranked(const uint32_t *perm, int64_t m, const int64_t *loff, const int64_t *at,
                        const uint32_t *lists, uint32_t *keys, uint32_t *vals, int64_t E, hipStream_t st)
{
    if (m <= 0) return;
    emit_ranked_kernel<<<grid_for((m + kEmitRanks - 1) / kEmitRanks, 1, 65535), 256, 0, st>>>(perm, m, loff, at, lists,
                                                                                              keys, vals, E);
    PCHECK_LAUNCH();
}

void launch_bucket_from_sorted(const Batch &b, const uint32_t *keys, const uint32_t *ents, int64_t E, int64_t P,
                               int64_t *bstart, uint32_t *bcnt, uint32_t *bmem, slot_t *bslot, int64_t *pos_of,
                               int64_t *bent, hipStream_t st)
{
    bucket_starts_kernel<<<grid_for(E + 1, 256), 256, 0, st>>>(keys, E, P, bstart);
    PCHECK_LAUNCH();
    bucket_counts_kernel<<<grid_for(P, 256), 256, 0, st>>>(bstart, P, bcnt);
    PCHECK_LAUNCH();
    if (E > 0) {
        bucket_members_kernel<<<grid_for(E, 256), 256, 0, st>>>(b, ents, E, bmem, bslot, pos_of, bent);
        PCHECK_LAUNCH();
    }
}

}  // namespace picasso
