// picasso_color_device_noalloc: the whole colouring of a small instance
// (every iteration of Alg. 1, in the one-workgroup tail kernel) with every
// intermediate buffer in a fixed device array, so that the call itself
// allocates no device memory.
//
// The array `scratch` below is the only memory the call uses beyond the
// caller's inputs and output.  Each device the library runs on holds its own
// copy until the process ends; its address on a device is taken once, with
// that device current, by hipGetSymbolAddress, and host code uses only that
// address (the array's name is not a device address on the host).  Every
// call on a device shares that device's copy, so calls that overlap on one
// device race; each call overwrites what it reads, clearing the padding flag
// with a fill kernel before use.
#include <cmath>
#include <mutex>
#include <vector>

#include "common.h"

namespace picasso {
namespace {

// Layout of the scratch array (offsets 256-byte aligned):
//   xz     kTailMax strings x 2W words (W <= 4), interleaved [x | z]
//   ids    kTailMax int32 (0 .. n-1)
//   table  (P, T) for 0..kTailMax vertices, 2 int32 each
//   rec    one TailRec
//   out    one TailOut
//   iters  kTailMax TailIter records
//   flag   int32 padding-violation flag
constexpr size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
constexpr size_t kOffXz = 0;
constexpr size_t kOffIds = kOffXz + align256((size_t)kTailMax * 8 * sizeof(uint64_t));
constexpr size_t kOffTable = kOffIds + align256((size_t)kTailMax * sizeof(int32_t));
constexpr size_t kOffRec = kOffTable + align256(2 * ((size_t)kTailMax + 1) * sizeof(int32_t));
constexpr size_t kOffOut = kOffRec + align256(sizeof(TailRec));
constexpr size_t kOffIters = kOffOut + align256(sizeof(TailOut));
constexpr size_t kOffFlag = kOffIters + align256((size_t)kTailMax * sizeof(TailIter));
constexpr size_t kScratchUsed = kOffFlag + align256(sizeof(int32_t));
constexpr size_t kScratchBytes = 64 << 10;
static_assert(kScratchUsed <= kScratchBytes, "scratch layout exceeds the array");
static_assert(kScratchBytes == PICASSO_NOALLOC_SCRATCH_BYTES && kTailMax == PICASSO_NOALLOC_MAX_N &&
                  kTailListCap == PICASSO_NOALLOC_MAX_LIST_ENTRIES,
              "the header's stated limits are the kernel's");

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The device address of the current device's scratch array, looked up once
// per device.
unsigned char *device_scratch()
{
    int dev = 0;
    PCHECK_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) throw Error(PICASSO_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        PCHECK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) throw Error(PICASSO_EDEVICE, "hipGetSymbolAddress returned a null scratch address");
        g_scratch_ptr[dev] = p;
    }
    return static_cast<unsigned char *>(g_scratch_ptr[dev]);
}

__global__ void noalloc_iota_kernel(int32_t *ids, int32_t n)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) ids[i] = i;
}

}  // namespace
}  // namespace picasso

using namespace picasso;

extern "C" int64_t picasso_color_device_noalloc(int64_t n, int32_t q, const uint64_t *x_words, const uint64_t *z_words,
                                                uint64_t seed, double palette_frac, double list_size, int32_t relation,
                                                int32_t *out_colors, void *stream)
{
    try {
        if (n < 0 || n > kTailMax)
            throw Error(PICASSO_EINVAL, "picasso_color_device_noalloc takes at most " + std::to_string(kTailMax) +
                                            " strings (got " + std::to_string(n) + ")");
        if (q < 1 || q > 256) throw Error(PICASSO_EINVAL, "q must be in [1, 256]");
        if (!(palette_frac > 0.0 && palette_frac <= 1.0)) throw Error(PICASSO_EINVAL, "palette_frac must be in (0, 1]");
        if (!(list_size > 0.0) || !std::isfinite(list_size)) throw Error(PICASSO_EINVAL, "list_size must be > 0");
        if (relation != PICASSO_REL_ANTICOMMUTE && relation != PICASSO_REL_QWC && relation != PICASSO_REL_COMMUTE)
            throw Error(PICASSO_EINVAL, "unknown relation");
        if (n > 0 && (!x_words || !z_words || !out_colors)) throw Error(PICASSO_EINVAL, "null pointer");
        if (n == 0) return 0;
        const int W = (q + 63) / 64;
        // (P, T) for every vertex count the iterations can reach, in host
        // double arithmetic (P = max(1, ceil(f m)), T = clamp(ceil(alpha ln m), 1, P)),
        // and the tail kernel's list capacity
        int32_t table[2 * (kTailMax + 1)] = {};
        for (int64_t k = 1; k <= n; ++k) {
            int64_t P = (int64_t)std::ceil(palette_frac * (double)k);
            if (P < 1) P = 1;
            int64_t T = (int64_t)std::ceil(list_size * std::log((double)k));
            if (T < 1) T = 1;
            if (T > P) T = P;
            if (T * k > kTailListCap)
                throw Error(PICASSO_EINVAL, "lists of " + std::to_string(T) + " colours for " + std::to_string(k) +
                                                " strings exceed the " + std::to_string(kTailListCap) +
                                                " list entries of picasso_color_device_noalloc");
            table[2 * k] = (int32_t)P;
            table[2 * k + 1] = (int32_t)T;
        }
        hipStream_t st = static_cast<hipStream_t>(stream);
        unsigned char *s = device_scratch();
        uint64_t *xz = reinterpret_cast<uint64_t *>(s + kOffXz);
        int32_t *ids = reinterpret_cast<int32_t *>(s + kOffIds);
        int32_t *d_table = reinterpret_cast<int32_t *>(s + kOffTable);
        TailRec *d_rec = reinterpret_cast<TailRec *>(s + kOffRec);
        TailOut *d_out = reinterpret_cast<TailOut *>(s + kOffOut);
        TailIter *d_iters = reinterpret_cast<TailIter *>(s + kOffIters);
        int32_t *flag = reinterpret_cast<int32_t *>(s + kOffFlag);
        // padding bits above q must be zero: checked before anything is written
        launch_fill_i32(flag, 1, 0, st);
        launch_check_padding(x_words, z_words, n, q, flag, st);
        int32_t bad = 0;
        PCHECK_HIP(hipMemcpyAsync(&bad, flag, sizeof(bad), hipMemcpyDeviceToHost, st));
        PCHECK_HIP(hipStreamSynchronize(st));
        if (bad) throw Error(PICASSO_EINVAL, "padding bits set");
        TailRec rec{};
        rec.src = 0;
        rec.m = n;
        rec.sbase = 0;
        rec.cbase = 0;
        rec.seed = seed;
        rec.ell = 1;
        rec.rel = relation;
        rec.table = 0;
        rec.iter0 = 0;
        PCHECK_HIP(hipMemcpyAsync(d_table, table, sizeof(int32_t) * 2 * ((size_t)n + 1), hipMemcpyHostToDevice, st));
        PCHECK_HIP(hipMemcpyAsync(d_rec, &rec, sizeof(rec), hipMemcpyHostToDevice, st));
        launch_interleave(x_words, z_words, n, W, xz, st);
        noalloc_iota_kernel<<<1, kTailMax, 0, st>>>(ids, (int32_t)n);
        PCHECK_LAUNCH();
        launch_tail(d_rec, 1, ids, xz, W, d_table, out_colors, d_out, d_iters, st);
        TailOut o{};
        PCHECK_HIP(hipMemcpyAsync(&o, d_out, sizeof(o), hipMemcpyDeviceToHost, st));
        PCHECK_HIP(hipStreamSynchronize(st));
        return o.n_colors;
    } catch (const Error &e) {
        set_last_error(e.what());
        return e.code;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return PICASSO_EINTERNAL;
    }
}
