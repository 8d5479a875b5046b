// Dynamic-order list colouring (Alg. 2, Sec. IV-B) in rounds.
//
// Alg. 2 takes one vertex at a time -- the one whose remaining list is
// shortest -- gives it a random colour of that list, and removes the colour
// from its neighbours' lists.  Here many vertices move per round:
//  1. active vertices (uncoloured, not failed) with an empty list fail; the
//     others are counted per instance by remaining list size;
//  2. per instance, R = max(ceil(A / divisor), min(A, 64)) of its A active
//     vertices request a colour: all with fewer than s* colours left (s* the
//     smallest size whose cumulative count reaches R) and those with exactly
//     s* whose keyed 32-bit draw falls below cut = floor(need 2^32 / eq);
//  3. a requester asks for a uniformly drawn entry of its remaining list;
//  4. in each colour bucket the requesters, in ascending (size, draw,
//     vertex) order, take the colour unless a relation neighbour in the
//     bucket took it first (requesters of a colour all hold it, so a
//     conflict edge between them is exactly a relation bit);
//  5. the bucket members related to a vertex that took the colour lose it.
// Steps 4 and 5 stay inside one bucket, so one wave per bucket does them
// from the bucket's relation rows (the matrix the static colouring uses),
// and only the rows of the bucket's requesters and winners are read: R is
// symmetric, so the members that lose the colour are the OR of the winners'
// rows.  Draws are keyed by (instance seed; vertex id in the instance,
// round, iteration, tag), so the result is that of the sequential
// description above, whatever the thread mapping.
#include <algorithm>

#include "common.h"

namespace picasso {
namespace {

constexpr int kWave = 64;
constexpr uint32_t TAG_DYNK = 0x44594E4Bu;  // request key
constexpr uint32_t TAG_DYNC = 0x44594E43u;  // requested entry
constexpr uint8_t DST_NONE = 0, DST_REQ = 1, DST_DEAD = 2;
constexpr int kHistThreads = 256;

// Step 1: failures, and per-instance counts of active vertices by remaining
// list size.  A block walks chunks of kHistThreads vertices; while its chunks
// lie in one instance it counts in LDS and adds the bins to the instance's
// global counters once (a large instance would otherwise put every block's
// bins, or every vertex, on a handful of global counters).
constexpr int kHistBlocks = 1024;
__global__ void __launch_bounds__(kHistThreads) dyn_hist_kernel(DynArgs a)
{
    extern __shared__ unsigned long long lh[];  // hist_w bins
    for (int i = threadIdx.x; i < a.hist_w; i += kHistThreads) lh[i] = 0ull;
    int32_t cur = -1;  // the instance the LDS bins count for (the same in every thread)
    auto flush = [&]() {
        __syncthreads();
        if (cur >= 0) {
            unsigned long long *g = a.hist + (int64_t)cur * a.hist_w;
            for (int i = threadIdx.x; i < a.hist_w; i += kHistThreads)
                if (lh[i]) {
                    atomicAdd(&g[i], lh[i]);
                    lh[i] = 0ull;
                }
        }
        __syncthreads();
    };
    __syncthreads();
    for (int64_t v0 = (int64_t)blockIdx.x * kHistThreads; v0 < a.m; v0 += (int64_t)gridDim.x * kHistThreads) {
        const int64_t v = v0 + threadIdx.x;
        const int64_t last = std::min<int64_t>(v0 + kHistThreads, a.m) - 1;
        const int32_t i0 = a.b.vinst[v0];
        const bool uniform = i0 == a.b.vinst[last];
        if (uniform && i0 != cur) {
            flush();
            cur = i0;
        }
        if (v < a.m && a.col[v] == COL_UNDECIDED) {
            const int32_t s = a.size[v];
            if (s == 0) {
                a.col[v] = COL_FAILED;
            } else if (uniform) {
                atomicAdd(&lh[s], 1ull);
            } else {
                atomicAdd(&a.hist[(int64_t)a.b.vinst[v] * a.hist_w + s], 1ull);
            }
        }
    }
    flush();
}

// Step 2: each instance's request threshold; the bins are cleared for the
// next round.  One workgroup; *active receives the number of active
// vertices of this round.
constexpr int kThrThreads = 256;
__global__ void __launch_bounds__(kThrThreads) dyn_threshold_kernel(DynArgs a)
{
    __shared__ unsigned long long wsum[kThrThreads / 64];
    unsigned long long total = 0;
    for (int32_t i = threadIdx.x; i < a.b.nb; i += kThrThreads) {
        unsigned long long *h = a.hist + (int64_t)i * a.hist_w;
        const int32_t T = a.b.inst[i].T;
        unsigned long long A = 0;
        for (int s = 1; s <= T; ++s) A += h[s];
        int32_t sstar = 0;
        uint64_t cut = 0;
        if (A > 0) {
            unsigned long long R = (A + a.divisor - 1) / a.divisor;
            const unsigned long long floor_r = A < 64 ? A : 64;
            if (R < floor_r) R = floor_r;
            unsigned long long below = 0, eq = 0;
            sstar = T;
            for (int s = 1; s <= T; ++s) {
                if (below + h[s] >= R) {
                    sstar = s;
                    eq = h[s];
                    break;
                }
                below += h[s];
            }
            const unsigned long long need = R - below;
            cut = need >= eq ? (1ull << 32) : (need << 32) / eq;
        }
        a.sstar[i] = sstar;
        a.cut[i] = cut;
        for (int s = 0; s <= T; ++s) h[s] = 0ull;
        total += A;
    }
    for (int d = 32; d > 0; d >>= 1) total += __shfl_down(total, d, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = total;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < kThrThreads / 64; ++w) t += wsum[w];
        *a.active = t;
    }
}

// Step 3: requests.  The requested entry is the j-th remaining slot in
// ascending slot (= colour) order; its bucket entry is flagged and the key
// (size, draw) kept for the bucket's ordering.
__global__ void dyn_request_kernel(DynArgs a, int32_t round)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < a.m; v += (int64_t)gridDim.x * blockDim.x) {
        if (a.col[v] != COL_UNDECIDED) continue;
        const int32_t s = a.size[v];
        if (s == 0) continue;
        const int32_t ii = a.b.vinst[v];
        const InstRec &r = a.b.inst[ii];
        const uint32_t vid = (uint32_t)(a.ids[v] - r.sbase);
        const uint64_t h = philox_draw(r.seed, vid, (uint32_t)round, a.ell, TAG_DYNK) >> 32;
        const int32_t sstar = a.sstar[ii];
        if (!(s < sstar || (s == sstar && h < a.cut[ii]))) continue;
        uint64_t j = __umul64hi(philox_draw(r.seed, vid, (uint32_t)round, a.ell, TAG_DYNC), (uint64_t)s);
        const uint64_t *al = a.alive + v * a.fw;
        int k = -1;
        for (int w = 0; w < a.fw; ++w) {
            uint64_t bits = al[w];
            const uint64_t cnt = (uint64_t)__popcll(bits);
            if (j >= cnt) {
                j -= cnt;
                continue;
            }
            for (; j > 0; --j) bits &= bits - 1;  // drop the j lowest set bits
            k = w * 64 + __builtin_ctzll(bits);
            break;
        }
        if (k < 0) continue;  // unreachable: j < size = set bits
        a.rkey[v] = ((uint64_t)s << 32) | h;
        a.st[a.pos_of[a.b.loff[v] + k]] = DST_REQ;
    }
}

// Steps 4 and 5: one wave per bucket.  The requesters are taken in key
// order (a wave-wide minimum over the bucket per pick; buckets hold few
// requesters per round); a requester whose relation row meets the winners
// so far is refused.  Then the winners' rows, OR-ed, mark the members that
// lose the colour.
__global__ void __launch_bounds__(kWave) dyn_resolve_kernel(DynArgs a)
{
    extern __shared__ uint64_t dl[];  // req[nw_max], acc[nw_max], lose[nw_max]
    uint64_t *req = dl, *acc = dl + a.nw_max, *lose = dl + 2 * a.nw_max;
    const int lane = threadIdx.x;
    for (int64_t c = blockIdx.x; c < a.P; c += gridDim.x) {
        const int64_t base = a.bstart[c];
        const int64_t S = a.bstart[c + 1] - base;
        const int64_t nw = (S + 63) >> 6;
        bool any = false;
        for (int64_t w = 0; w < nw; ++w) {
            const int64_t p = w * kWave + lane;
            const bool r = p < S && a.st[base + p] == DST_REQ;
            const uint64_t bal = __ballot(r);
            if (lane == 0) {
                req[w] = bal;
                acc[w] = 0ull;
                lose[w] = 0ull;
            }
            any |= bal != 0ull;
        }
        if (!any) continue;  // wave-uniform
        __syncthreads();
        const uint64_t *Rm = a.R + a.rb_off[c];
        while (true) {
            // the requester with the smallest (key, vertex)
            uint64_t bk = ~0ull;
            uint32_t bv = 0xFFFFFFFFu;
            int64_t bp = -1;
            for (int64_t w = 0; w < nw; ++w) {
                const uint64_t rw = req[w];
                if (!rw) continue;
                if ((rw >> lane) & 1ull) {
                    const int64_t p = w * kWave + lane;
                    const uint32_t v = a.bmem[base + p];
                    const uint64_t k = a.rkey[v];
                    if (k < bk || (k == bk && v < bv)) {
                        bk = k;
                        bv = v;
                        bp = p;
                    }
                }
            }
            for (int d = 32; d > 0; d >>= 1) {
                const uint64_t ok = __shfl_xor(bk, d, 64);
                const uint32_t ov = __shfl_xor(bv, d, 64);
                const int64_t op = __shfl_xor(bp, d, 64);
                if (ok < bk || (ok == bk && ov < bv)) {
                    bk = ok;
                    bv = ov;
                    bp = op;
                }
            }
            if (bp < 0) break;  // wave-uniform: no requester left
            // refused if its relation row meets a winner
            const uint64_t *row = Rm + bp * nw;
            bool hit = false;
            for (int64_t w = lane; w < nw; w += kWave) hit |= (row[w] & acc[w]) != 0ull;
            const bool refused = __ballot(hit) != 0ull;
            __syncthreads();
            if (lane == 0) {
                req[bp >> 6] &= ~(1ull << (bp & 63));
                a.st[base + bp] = DST_NONE;
                if (!refused) {
                    acc[bp >> 6] |= 1ull << (bp & 63);
                    a.col[bv] = (int32_t)c;
                }
            }
            if (!refused)
                for (int64_t w = lane; w < nw; w += kWave) lose[w] |= row[w];
            __syncthreads();
        }
        // members related to a winner lose the colour (winners excluded; a
        // member may be coloured elsewhere already, which is harmless)
        for (int64_t w = 0; w < nw; ++w) {
            const int64_t p = w * kWave + lane;
            const uint64_t bits = lose[w] & ~acc[w];
            if (p < S && ((bits >> lane) & 1ull)) {
                if (a.st[base + p] != DST_DEAD) {
                    a.st[base + p] = DST_DEAD;
                    const uint32_t v = a.bmem[base + p];
                    const int k = a.bslot[base + p];
                    atomicAnd((unsigned long long *)&a.alive[(int64_t)v * a.fw + (k >> 6)], ~(1ull << (k & 63)));
                    atomicSub(&a.size[v], 1);
                }
            }
        }
        __syncthreads();
    }
}

// Initial state: every slot of a vertex alive, size T_v, colour undecided.
__global__ void dyn_init_kernel(DynArgs a)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < a.m; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t T = (int32_t)(a.b.loff[v + 1] - a.b.loff[v]);
        for (int w = 0; w < a.fw; ++w) {
            const int lo = w * 64;
            uint64_t bits = 0ull;
            if (T >= lo + 64) bits = ~0ull;
            else if (T > lo) bits = (1ull << (T - lo)) - 1ull;
            a.alive[v * a.fw + w] = bits;
        }
        a.size[v] = T;
        a.col[v] = COL_UNDECIDED;
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

void launch_dyn_init(const DynArgs &a, hipStream_t st)
{
    if (a.m <= 0) return;
    dyn_init_kernel<<<grid_for(a.m, 256), 256, 0, st>>>(a);
    PCHECK_LAUNCH();
}

void launch_dyn_round(const DynArgs &a, int32_t round, hipStream_t st)
{
    if (a.m <= 0) return;
    const int64_t hb = (a.m + kHistThreads - 1) / kHistThreads;
    if (hb > 0x7FFFFFFF) throw Error(PICASSO_EINTERNAL, "dynamic colouring: too many vertices");
    dyn_hist_kernel<<<(unsigned)std::min<int64_t>(hb, kHistBlocks), kHistThreads,
                      (size_t)a.hist_w * sizeof(unsigned long long), st>>>(a);
    PCHECK_LAUNCH();
    dyn_threshold_kernel<<<1, kThrThreads, 0, st>>>(a);
    PCHECK_LAUNCH();
    dyn_request_kernel<<<grid_for(a.m, 256), 256, 0, st>>>(a, round);
    PCHECK_LAUNCH();
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(a.P, 16384));
    dyn_resolve_kernel<<<(unsigned)grid, kWave, (size_t)3 * a.nw_max * sizeof(uint64_t), st>>>(a);
    PCHECK_LAUNCH();
}

}  // namespace picasso
