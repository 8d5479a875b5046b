// List colouring of the conflict graph in a random static order
// (Sec. IV-B, static order schemes; Alg. 1 colour step) and the hand-over
// to the next iteration (Alg. 1: recurse on the uncoloured vertices with a
// fresh palette).
//
// Sequential rule: take the vertices by ascending (priority, index); each
// takes the smallest colour of its list that no earlier neighbour holds, or
// stays uncoloured.  Jones-Plassmann evaluates the same rule in parallel: a
// vertex is decided once every earlier neighbour is decided, so its choice
// sees exactly the colours the sequential order would have shown it.
//
// Each vertex keeps a cursor into its CSR row: earlier neighbours already
// seen decided are never re-read, their colours accumulated into a bit
// mask over the vertex's list slots.
#include "common.h"

namespace picasso {
namespace {

__device__ __forceinline__ bool earlier(uint64_t pj, int64_t j, uint64_t pi, int64_t i)
{
    return pj < pi || (pj == pi && j < i);
}

__device__ __forceinline__ int32_t load_col(const int32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void color_init_kernel(ColorArgs a)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.m; i += (int64_t)gridDim.x * blockDim.x) {
        a.col[i] = COL_UNDECIDED;
        a.cursor[i] = a.rowptr[i];
        for (int w = 0; w < a.fw; ++w) a.forbid[i * a.fw + w] = 0;
    }
}

__global__ void color_round_kernel(ColorArgs a)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.m; i += (int64_t)gridDim.x * blockDim.x) {
        if (load_col(&a.col[i]) != COL_UNDECIDED) continue;
        const uint64_t pi = a.prio[i];
        const uint32_t *Li = a.lists + i * a.T;
        const int64_t end = a.rowptr[i + 1];
        int64_t e = a.cursor[i];
        for (; e < end; ++e) {
            const int64_t j = a.adj[e];
            if (!earlier(a.prio[j], j, pi, i)) continue;
            const int32_t cj = load_col(&a.col[j]);
            if (cj == COL_UNDECIDED) break;
            if (cj < 0) continue;  // failed neighbour holds no colour
            int lo = 0, hi = a.T;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (Li[mid] < (uint32_t)cj) lo = mid + 1;
                else hi = mid;
            }
            if (lo < a.T && Li[lo] == (uint32_t)cj) a.forbid[i * a.fw + (lo >> 6)] |= 1ull << (lo & 63);
        }
        a.cursor[i] = e;
        if (e < end) continue;
        int32_t pick = COL_FAILED;
        for (int w = 0; w < a.fw; ++w) {
            const uint64_t freebits = ~a.forbid[i * a.fw + w];
            if (freebits) {
                const int slot = w * 64 + __builtin_ctzll(freebits);
                if (slot < a.T) pick = (int32_t)Li[slot];
                break;
            }
        }
        __hip_atomic_store(&a.col[i], pick, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        atomicAdd(a.progress, 1ull);
    }
}

__global__ void finish_kernel(int64_t m, const int32_t *col, const int32_t *ids, int64_t offset,
                              int32_t *out_colors, uint32_t *used_bits, unsigned long long *n_used,
                              int32_t *uncol_flag)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t c = col[i];
        if (c >= 0) {
            out_colors[ids[i]] = (int32_t)(offset + c);
            const uint32_t bit = 1u << (c & 31);
            if (!(atomicOr(&used_bits[c >> 5], bit) & bit)) atomicAdd(n_used, 1ull);
            uncol_flag[i] = 0;
        } else {
            uncol_flag[i] = 1;
        }
    }
}

__global__ void compact_kernel(int64_t m, const int32_t *ids, const int32_t *flag, const int64_t *pos,
                               int32_t *next_ids)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        if (flag[i]) next_ids[pos[i]] = ids[i];
}

unsigned grid_for(int64_t work, int threads)
{
    int64_t b = (work + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > 65535 * 16) b = 65535 * 16;
    return (unsigned)b;
}

}  // namespace

void launch_color_init(const ColorArgs &a, hipStream_t st)
{
    if (a.m <= 0) return;
    color_init_kernel<<<grid_for(a.m, 256), 256, 0, st>>>(a);
    PCHECK_LAUNCH();
}

void launch_color_round(const ColorArgs &a, hipStream_t st)
{
    if (a.m <= 0) return;
    color_round_kernel<<<grid_for(a.m, 256), 256, 0, st>>>(a);
    PCHECK_LAUNCH();
}

void launch_finish_iteration(int64_t m, const int32_t *col, const int32_t *ids, int64_t offset, int32_t *out_colors,
                             uint32_t *used_bits, unsigned long long *n_used, int32_t *uncol_flag, hipStream_t st)
{
    if (m <= 0) return;
    finish_kernel<<<grid_for(m, 256), 256, 0, st>>>(m, col, ids, offset, out_colors, used_bits, n_used, uncol_flag);
    PCHECK_LAUNCH();
}

void launch_compact_ids(int64_t m, const int32_t *ids, const int32_t *flag, const int64_t *pos, int32_t *next_ids,
                        hipStream_t st)
{
    if (m <= 0) return;
    compact_kernel<<<grid_for(m, 256), 256, 0, st>>>(m, ids, flag, pos, next_ids);
    PCHECK_LAUNCH();
}

}  // namespace picasso
