// The last iterations of Alg. 1 for an instance with few uncoloured
// vertices, all on the device in one workgroup.
//
// Once an instance has at most kTailMax vertices left, each further
// iteration is tiny but would still cost the full sequence of launches and
// host round trips.  Here one workgroup per instance runs every remaining
// iteration in LDS: lists (Floyd, the same keyed Philox draws as the list
// kernel), priorities, the vertices sorted by (priority, index), and the
// sequential list greedy in that order (Sec. IV-B, static order): each vertex
// takes the smallest colour of its list that no earlier conflicting vertex
// holds.  An earlier vertex u matters only if it holds a colour c of v's
// list, and then u and v share c, so u conflicts with v exactly when the
// relation holds: the greedy needs the relation bits and the colours, not
// the conflict graph.  The per-iteration sizes the statistics report
// (pair tests, conflict edges) are counted alongside.  Palette and list
// sizes come from a table the host fills with its own double arithmetic.
#include "common.h"

namespace picasso {
namespace {

constexpr int kTailThreads = 256;

__device__ __forceinline__ bool tail_relation(const uint64_t *su, const uint64_t *sv, int W, int rel)
{
    uint64_t par = 0, any = 0;
    for (int w = 0; w < W; ++w) {
        const uint64_t t = (su[w] & sv[W + w]) ^ (su[W + w] & sv[w]);
        par ^= t;
        any |= t;
    }
    if (rel == PICASSO_REL_ANTICOMMUTE) return __popcll(par) & 1;
    if (rel == PICASSO_REL_COMMUTE) return !(__popcll(par) & 1);
    return any != 0;
}

__global__ void __launch_bounds__(kTailThreads) tail_kernel(const TailRec *__restrict__ recs,
                                                            const int32_t *__restrict__ ids,
                                                            const uint64_t *__restrict__ xz, int32_t W,
                                                            const int32_t *__restrict__ table,
                                                            int32_t *__restrict__ out_colors,
                                                            TailOut *__restrict__ outs, TailIter *__restrict__ iters)
{
    __shared__ uint64_t str[kTailMax * 2 * 4];     // member strings [x | z], W <= 4
    __shared__ uint8_t lists[kTailListCap];         // m x T colours (P <= kTailMax)
    __shared__ uint32_t rel[kTailMax * kTailMax / 32];  // relation bits, row u: bit v
    __shared__ int32_t vid[kTailMax];               // instance-local vertex id (ascending)
    __shared__ uint64_t prio[kTailMax];
    __shared__ int32_t order[kTailMax];             // vertices in colouring order
    __shared__ int32_t col[kTailMax];               // palette colour, -1 uncoloured
    __shared__ int32_t cnt[kTailMax];               // bucket sizes
    __shared__ int32_t flag[kTailMax + 1];
    __shared__ unsigned long long acc[2];           // pair tests, edges
    __shared__ int used_n, m_sh;
    const TailRec r = recs[blockIdx.x];
    const int t = threadIdx.x;
    int m = (int)r.m;
    for (int i = t; i < m; i += kTailThreads) {
        const int64_t g = ids[r.src + i];
        vid[i] = (int32_t)(g - r.sbase);
        for (int w = 0; w < 2 * W; ++w) str[i * 2 * W + w] = xz[g * 2 * W + w];
    }
    int64_t cbase = r.cbase;
    uint32_t ell = (uint32_t)r.ell;
    int n_iters = 0;
    int64_t n_used_total = 0;
    __syncthreads();
    while (m > 0) {
        const int P = table[r.table + 2 * m], T = table[r.table + 2 * m + 1];
        // lists and priorities
        for (int i = t; i < m; i += kTailThreads) {
            uint8_t *s = lists + i * T;
            for (int step = 0; step < T; ++step) {
                const uint64_t j = (uint64_t)(P - T + step);
                const uint64_t rnd = philox_draw(r.seed, (uint32_t)vid[i], (uint32_t)step, ell, TAG_LIST);
                const uint32_t cand = (uint32_t)__umul64hi(rnd, j + 1);
                int lo = 0, hi = step;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (s[mid] < cand) lo = mid + 1;
                    else hi = mid;
                }
                if (lo < step && s[lo] == cand) {
                    s[step] = (uint8_t)j;
                } else {
                    for (int k = step; k > lo; --k) s[k] = s[k - 1];
                    s[lo] = (uint8_t)cand;
                }
            }
            prio[i] = philox_draw(r.seed, (uint32_t)vid[i], 0, ell, TAG_PRIO);
            order[i] = i;
            col[i] = -1;
        }
        for (int c = t; c < P; c += kTailThreads) cnt[c] = 0;
        if (t < 2) acc[t] = 0ull;
        if (t == 0) used_n = 0;
        __syncthreads();
        // relation bits, bucket sizes, conflict edges
        const int rw = (m + 31) >> 5;
        for (int idx = t; idx < m * rw; idx += kTailThreads) {
            const int u = idx / rw, w = idx - u * rw;
            uint32_t bits = 0u;
            for (int b = 0; b < 32; ++b) {
                const int v = w * 32 + b;
                if (v < m && v != u && tail_relation(str + u * 2 * W, str + v * 2 * W, W, r.rel)) bits |= 1u << b;
            }
            rel[u * rw + w] = bits;
        }
        for (int e = t; e < m * T; e += kTailThreads) atomicAdd(&cnt[lists[e]], 1);
        __syncthreads();
        unsigned long long tests = 0, edges = 0;
        for (int c = t; c < P; c += kTailThreads) tests += (unsigned long long)cnt[c] * (cnt[c] - 1) / 2;
        for (int idx = t; idx < m * m; idx += kTailThreads) {
            const int u = idx / m, v = idx - u * m;
            if (u >= v || !((rel[u * rw + (v >> 5)] >> (v & 31)) & 1u)) continue;
            const uint8_t *Lu = lists + u * T, *Lv = lists + v * T;
            int x = 0, y = 0;
            while (x < T && y < T) {
                if (Lu[x] == Lv[y]) {
                    ++edges;
                    break;
                }
                if (Lu[x] < Lv[y]) ++x;
                else ++y;
            }
        }
        if (tests) atomicAdd(&acc[0], tests);
        if (edges) atomicAdd(&acc[1], edges);
        // colouring order: bitonic sort of (priority, index) over a power of
        // two, padded with entries of the largest key
        int N = 1;
        while (N < m) N <<= 1;
        for (int i = m + t; i < N; i += kTailThreads) {
            order[i] = i;
            prio[i] = ~0ull;
        }
        for (int k = 2; k <= N; k <<= 1)
            for (int j = k >> 1; j > 0; j >>= 1) {
                __syncthreads();
                for (int e = t; e < N; e += kTailThreads) {
                    const int f = e ^ j;
                    if (f > e) {
                        const int a = order[e], b = order[f];
                        const bool gt = prio[a] > prio[b] || (prio[a] == prio[b] && a > b);
                        if (gt == ((e & k) == 0)) {
                            order[e] = b;
                            order[f] = a;
                        }
                    }
                }
            }
        __syncthreads();
        // sequential greedy in that order, run by one wave (no workgroup
        // barrier per vertex): for each vertex the lanes scan the earlier
        // vertices, the colours held by conflicting ones are OR-reduced, and
        // a ballot over the list slots picks the first colour not held
        if (t < 64) {
            const int lane = t;
            for (int i = 0; i < m; ++i) {
                const int v = order[i];
                uint64_t f[kTailMax / 64];
#pragma unroll
                for (int w = 0; w < kTailMax / 64; ++w) f[w] = 0ull;
                for (int j = lane; j < i; j += 64) {
                    const int u = order[j];
                    const int cu = col[u];
                    if (cu >= 0 && ((rel[v * rw + (u >> 5)] >> (u & 31)) & 1u)) {
#pragma unroll
                        for (int w = 0; w < kTailMax / 64; ++w)
                            if ((cu >> 6) == w) f[w] |= 1ull << (cu & 63);
                    }
                }
#pragma unroll
                for (int w = 0; w < kTailMax / 64; ++w)
                    for (int d = 32; d > 0; d >>= 1) f[w] |= __shfl_xor(f[w], d, 64);
                int take = -1;
                for (int k0 = 0; k0 < T && take < 0; k0 += 64) {
                    const int k = k0 + lane;
                    bool free_slot = false;
                    if (k < T) {
                        const int c = lists[v * T + k];
                        uint64_t fw = 0ull;
#pragma unroll
                        for (int w = 0; w < kTailMax / 64; ++w)
                            if ((c >> 6) == w) fw = f[w];
                        free_slot = !((fw >> (c & 63)) & 1ull);
                    }
                    const uint64_t ok = __ballot(free_slot);
                    if (ok) take = lists[v * T + k0 + __builtin_ctzll(ok)];
                }
                if (lane == 0) col[v] = take;
                // the colour is in LDS before any lane reads it for a later vertex
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
        }
        __syncthreads();
        // outputs, used colours, next vertex set (ascending ids kept)
        for (int c = t; c < P; c += kTailThreads) cnt[c] = 0;
        __syncthreads();
        for (int i = t; i < m; i += kTailThreads) {
            const int c = col[i];
            if (c >= 0) {
                out_colors[r.sbase + vid[i]] = (int32_t)(cbase + c);
                if (atomicExch(&cnt[c], 1) == 0) atomicAdd(&used_n, 1);
            }
            flag[i] = c < 0;
        }
        __syncthreads();
        if (t == 0) {
            int s = 0;
            for (int i = 0; i < m; ++i) {
                const int f = flag[i];
                flag[i] = s;
                s += f;
            }
            flag[m] = s;
            m_sh = s;
            TailIter it;
            it.m = m;
            it.P = P;
            it.T = T;
            it.pair_tests = (int64_t)acc[0];
            it.edges = (int64_t)acc[1];
            it.colored = m - s;
            it.offset = cbase;
            iters[r.iter0 + n_iters] = it;
            n_used_total += used_n;
        }
        __syncthreads();
        // compact vertex ids and strings in place (destination index <= source index)
        const int m_next = m_sh;
        for (int base = 0; base < m; base += kTailThreads) {
            const int i = base + t;
            int32_t keep_vid = 0;
            uint64_t keep[8];
            bool keep_it = false;
            int dst = 0;
            if (i < m && col[i] < 0) {
                keep_it = true;
                dst = flag[i];
                keep_vid = vid[i];
                for (int w = 0; w < 2 * W; ++w) keep[w] = str[i * 2 * W + w];
            }
            __syncthreads();
            if (keep_it) {
                vid[dst] = keep_vid;
                for (int w = 0; w < 2 * W; ++w) str[dst * 2 * W + w] = keep[w];
            }
            __syncthreads();
        }
        cbase += P;
        ++ell;
        ++n_iters;
        m = m_next;
        if (t == 0) used_n = 0;
        __syncthreads();
    }
    if (t == 0) {
        TailOut o;
        o.n_colors = n_used_total;
        o.n_iters = n_iters;
        outs[blockIdx.x] = o;
    }
}

__global__ void gather_ranges_kernel(const int32_t *__restrict__ src, int32_t *__restrict__ dst,
                                     const int64_t *__restrict__ ranges, int32_t nr, int64_t total)
{
    // ranges: nr x (src start, dst start), ascending dst start; range r covers
    // dst [dst_r, dst_{r+1}) (the last one up to total)
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < total; j += (int64_t)gridDim.x * blockDim.x) {
        int lo = 0, hi = nr;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (ranges[2 * mid + 1] <= j) lo = mid;
            else hi = mid;
        }
        dst[j] = src[ranges[2 * lo] + (j - ranges[2 * lo + 1])];
    }
}

}  // namespace

void launch_tail(const TailRec *recs, int32_t n, const int32_t *ids, const uint64_t *xz, int32_t W,
                 const int32_t *table, int32_t *out_colors, TailOut *outs, TailIter *iters, hipStream_t st)
{
    if (n <= 0) return;
    if (W > 4) throw Error(PICASSO_EINTERNAL, "tail: unsupported word count");
    tail_kernel<<<(unsigned)n, kTailThreads, 0, st>>>(recs, ids, xz, W, table, out_colors, outs, iters);
    PCHECK_LAUNCH();
}

void launch_gather_ranges(const int32_t *src, int32_t *dst, const int64_t *ranges, int32_t nr, int64_t total,
                          hipStream_t st)
{
    if (total <= 0 || nr <= 0) return;
    int64_t b = (total + 255) / 256;
    if (b > 65535 * 16) b = 65535 * 16;
    gather_ranges_kernel<<<(unsigned)b, 256, 0, st>>>(src, dst, ranges, nr, total);
    PCHECK_LAUNCH();
}

}  // namespace picasso
