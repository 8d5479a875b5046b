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
void launch_sample_lists(uint64_t seed, uint32_t ell, int64_t m, const int32_t *ids, int64_t P, int32_t T,
                         uint32_t *lists, uint64_t *prio, hipStream_t st);
void launch_bucket_count(const uint32_t *lists, int64_t entries, uint32_t *bcnt, hipStream_t st);
void launch_bucket_scatter(const uint32_t *lists, int64_t m, int32_t T, const int64_t *bstart, uint32_t *bfill,
                           uint32_t *bmem, uint8_t *bslot, hipStream_t st);
void launch_check_padding(const uint64_t *x, const uint64_t *z, int64_t n, int32_t q, int32_t *bad,
                          hipStream_t st);

// pairs.hip: the intra-bucket pair kernels.
struct PairArgs {
    const int64_t *bstart;  // [P+1]
    const uint32_t *bmem;   // local vertex index of each bucket entry
    const uint8_t *bslot;   // slot of the bucket colour in that vertex's list
    int64_t P;
    const int32_t *ids;     // local -> original id
    const uint64_t *x, *z;  // all n strings, n x W
    int32_t W;
    const uint32_t *lists;  // m x T, rows sorted
    int32_t T;
    int32_t relation;
    int64_t m;
    // count pass
    int32_t *deg;
    // fill pass
    const int64_t *rowptr;
    int32_t *cursor;
    int32_t *adj;
};
void launch_pair_count(const PairArgs &a, hipStream_t st);
void launch_pair_fill(const PairArgs &a, hipStream_t st);

// color.hip
struct ColorArgs {
    int64_t m;
    const int64_t *rowptr;
    const int32_t *adj;
    const uint64_t *prio;
    const uint32_t *lists;
    int32_t T;
    int32_t *col;       // local palette colour, -1 failed, -2 undecided
    int64_t *cursor;    // per-vertex resume position in its row
    uint64_t *forbid;   // m x FW words, bit k = slot k taken by an earlier neighbour
    int32_t fw;         // words per forbid mask = ceil(T/64)
    unsigned long long *progress;  // count of decided vertices
};
void launch_color_init(const ColorArgs &a, hipStream_t st);
void launch_color_round(const ColorArgs &a, hipStream_t st);
void launch_finish_iteration(int64_t m, const int32_t *col, const int32_t *ids, int64_t offset, int32_t *out_colors,
                             uint32_t *used_bits, unsigned long long *n_used, int32_t *uncol_flag, hipStream_t st);
void launch_bucket_pairs(const uint32_t *bcnt, int64_t P, unsigned long long *pairs, hipStream_t st);
void launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t st);
void launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t st);
void launch_compact_ids(int64_t m, const int32_t *ids, const int32_t *flag, const int64_t *pos, int32_t *next_ids,
                        hipStream_t st);

}  // namespace picasso
