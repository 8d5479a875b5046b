// Exclusive prefix sums (reduce-then-scan over 2048-element tiles).
//
// Used for the bucket offsets (colour-bucket build), the CSR row pointer
// (Alg. 3's exclusive sum over per-vertex edge counts) and the compaction
// of the uncoloured vertex set (Alg. 1, next iteration's vertices).
#include "common.h"

namespace picasso {
namespace {

constexpr int kThreads = 256;
constexpr int kItems = 8;
constexpr int64_t kTile = (int64_t)kThreads * kItems;

__device__ __forceinline__ int64_t wave_inclusive_scan(int64_t v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int64_t o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

// Exclusive scan of one value per thread across the block; returns the
// thread's exclusive prefix and writes the block total to *total.
__device__ __forceinline__ int64_t block_exclusive_scan(int64_t v, int64_t *total)
{
    __shared__ int64_t wsum[kThreads / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int64_t inc = wave_inclusive_scan(v);
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    int64_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) {
        if (w < wave) before += wsum[w];
        all += wsum[w];
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

template <typename In>
__global__ void __launch_bounds__(kThreads) tile_reduce(const In *in, int64_t n, int64_t *partial)
{
    const int64_t base = (int64_t)blockIdx.x * kTile;
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t i = base + (int64_t)k * kThreads + threadIdx.x;
        if (i < n) s += (int64_t)in[i];
    }
    int64_t total;
    block_exclusive_scan(s, &total);
    if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

template <typename In>
__global__ void __launch_bounds__(kThreads) tile_scan(const In *in, int64_t n, const int64_t *offsets, int64_t *out,
                                                      bool with_total)
{
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
    int64_t v[kItems];
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t i = base + k;
        v[k] = i < n ? (int64_t)in[i] : 0;
        s += v[k];
    }
    int64_t total;
    int64_t run = block_exclusive_scan(s, &total) + (offsets ? offsets[blockIdx.x] : 0);
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t i = base + k;
        if (i < n) out[i] = run;
        run += v[k];
    }
    if (with_total && blockIdx.x == gridDim.x - 1 && threadIdx.x == kThreads - 1) out[n] = run;
}

int64_t tiles(int64_t n) { return (n + kTile - 1) / kTile; }

__global__ void zero_one(int64_t *p) { *p = 0; }

template <typename In>
void scan_impl(const In *in, int64_t *out, int64_t n, bool with_total, char *tmp, hipStream_t st)
{
    if (n <= 0) {
        if (with_total) {
            zero_one<<<1, 1, 0, st>>>(out);
            PCHECK_LAUNCH();
        }
        return;
    }
    const int64_t nb = tiles(n);
    if (nb == 1) {
        tile_scan<In><<<1, kThreads, 0, st>>>(in, n, nullptr, out, with_total);
        PCHECK_LAUNCH();
        return;
    }
    int64_t *partial = reinterpret_cast<int64_t *>(tmp);
    int64_t *offsets = partial + ((nb + 63) / 64) * 64;
    tile_reduce<In><<<(unsigned)nb, kThreads, 0, st>>>(in, n, partial);
    PCHECK_LAUNCH();
    scan_impl<int64_t>(partial, offsets, nb, false, reinterpret_cast<char *>(offsets + ((nb + 63) / 64) * 64), st);
    tile_scan<In><<<(unsigned)nb, kThreads, 0, st>>>(in, n, offsets, out, with_total);
    PCHECK_LAUNCH();
}

}  // namespace

size_t scan_tmp_bytes(int64_t n)
{
    size_t bytes = 0;
    while (n > kTile) {
        const int64_t nb = tiles(n);
        bytes += 2 * (size_t)((nb + 63) / 64) * 64 * sizeof(int64_t);
        n = nb;
    }
    return bytes + 256;
}

void exclusive_scan_u32_to_i64(const uint32_t *in, int64_t *out, int64_t n, bool with_total, void *tmp,
                               hipStream_t st)
{
    scan_impl<uint32_t>(in, out, n, with_total, static_cast<char *>(tmp), st);
}

void exclusive_scan_i32_to_i64(const int32_t *in, int64_t *out, int64_t n, bool with_total, void *tmp,
                               hipStream_t st)
{
    scan_impl<int32_t>(in, out, n, with_total, static_cast<char *>(tmp), st);
}

void exclusive_scan_i64(const int64_t *in, int64_t *out, int64_t n, bool with_total, void *tmp, hipStream_t st)
{
    scan_impl<int64_t>(in, out, n, with_total, static_cast<char *>(tmp), st);
}

}  // namespace picasso
