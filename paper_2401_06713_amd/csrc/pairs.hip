// Intra-bucket pair kernels: the conflict-graph build (Alg. 1
// construct_conflict_graph; Sec. IV-A; the CSR output of Alg. 3).
//
// A pair {u, v} conflicts iff the relation holds and L(u), L(v) share a
// colour.  Such a pair lies in the bucket of each shared colour; it is kept
// once, in the bucket of its smallest shared colour c.  Lists are sorted, so
// "no smaller shared colour" means the list prefixes before c are disjoint.
//
// Relation, popcount form: with a = (x_u & z_v) ^ (z_u & x_v), bit k of a is
// set exactly when position k holds two different non-identity Paulis
// (Eq. 5).  ANTICOMMUTE: parity of popcount(a) (the parity rule of
// Sec. IV-A); QWC: a != 0.
//
// Buckets are sorted by vertex priority, so member order is the colouring
// order.  Per bucket the kernels keep two S x S bit matrices in HBM, row p
// holding ceil(S/64) words:
//   R: relation bits between members (symmetric), written by relate_kernel;
//   D: pairs that share a colour smaller than the bucket's (dup_kernel).
// The bucket's conflict edges are R & ~D.  count_kernel pop-counts each
// row into the member's (vertex, slot) segment length; after a scan,
// fill_kernel expands each row into its CSR segment.  The colouring reads
// the lower triangle of R (earlier members) directly.
#include "common.h"

namespace picasso {
namespace {

constexpr int kWave = 64;

// Bucket index owning work item `item`, given offsets off[0..P] (off[P] =
// total items): the largest c with off[c] <= item.
__device__ __forceinline__ int64_t find_bucket(const int64_t *__restrict__ off, int64_t P, int64_t item)
{
    int64_t lo = 0, hi = P;  // off[lo] <= item < off[hi]
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (off[mid] <= item) lo = mid;
        else hi = mid;
    }
    return lo;
}

template <int W, int REL>
__device__ __forceinline__ uint32_t pair_bit(const uint32_t (&xi)[2 * W], const uint32_t (&zi)[2 * W],
                                             const uint32_t *xj, const uint32_t *zj)
{
    uint32_t acc = 0;
#pragma unroll
    for (int h = 0; h < 2 * W; ++h) {
        const uint32_t a = (xi[h] & zj[h]) ^ (zi[h] & xj[h]);
        if (REL == PICASSO_REL_ANTICOMMUTE) acc ^= a;
        else acc |= a;
    }
    if (REL == PICASSO_REL_ANTICOMMUTE) return __popc(acc) & 1u;
    return acc != 0u;
}

// 64 x 64 bit transpose across a wave: lane l holds row l; afterwards lane
// l holds column l (bit j = old bit l of lane j).
__device__ __forceinline__ uint64_t wave_transpose64(uint64_t r)
{
    const int lane = threadIdx.x & 63;
    {  // s = 32: swap the high half of lanes 0..31 with the low half of lanes 32..63
        uint32_t lo = (uint32_t)r, hi = (uint32_t)(r >> 32);
        const uint32_t send = (lane & 32) ? lo : hi;
        const uint32_t got = (uint32_t)__shfl_xor((int)send, 32, 64);
        if (lane & 32) lo = got;
        else hi = got;
        r = ((uint64_t)hi << 32) | lo;
    }
    const uint64_t masks[5] = {0x0000FFFF0000FFFFull, 0x00FF00FF00FF00FFull, 0x0F0F0F0F0F0F0F0Full,
                               0x3333333333333333ull, 0x5555555555555555ull};
#pragma unroll
    for (int t = 0; t < 5; ++t) {
        const int s = 16 >> t;
        const uint64_t m = masks[t];
        const uint32_t plo = (uint32_t)__shfl_xor((int)(uint32_t)r, s, 64);
        const uint32_t phi = (uint32_t)__shfl_xor((int)(uint32_t)(r >> 32), s, 64);
        const uint64_t p = ((uint64_t)phi << 32) | plo;
        if (lane & s) r = (r & ~m) | ((p & ~m) >> s);
        else r = (r & m) | ((p & m) << s);
    }
    return r;
}

// One wave per (bucket, row tile of 64 members).  Row members stay in
// registers; each column tile (64 members, zero-padded) is staged in LDS and
// read by broadcast.  Lane i accumulates the relation bits of row i against
// the tile's 64 columns; a bit transpose turns the tile into the column
// members' words, so each tile is tested once and written twice.
template <int W, int REL>
__global__ void __launch_bounds__(kWave) relate_kernel(RelateArgs a)
{
    __shared__ uint32_t cx[kWave * 2 * W], cz[kWave * 2 * W];
    const int lane = threadIdx.x;
    for (int64_t item = blockIdx.x; item < a.total_row_tiles; item += gridDim.x) {
        const int64_t c = find_bucket(a.tile_off, a.P, item);
        const int64_t rt = item - a.tile_off[c];
        const int64_t base = a.bstart[c];
        const int64_t S = a.bstart[c + 1] - base;
        const int64_t nw = (S + 63) >> 6;
        uint64_t *Rm = a.R + a.rb_off[c];
        const int64_t i = rt * kWave + lane;
        uint32_t xi[2 * W], zi[2 * W];
        if (i < S) {
            const int64_t g = (int64_t)a.ids[a.bmem[base + i]] * W;
#pragma unroll
            for (int w = 0; w < W; ++w) {
                const uint64_t xv = a.x[g + w], zv = a.z[g + w];
                xi[2 * w] = (uint32_t)xv;
                xi[2 * w + 1] = (uint32_t)(xv >> 32);
                zi[2 * w] = (uint32_t)zv;
                zi[2 * w + 1] = (uint32_t)(zv >> 32);
            }
        } else {
#pragma unroll
            for (int h = 0; h < 2 * W; ++h) xi[h] = zi[h] = 0u;
        }
        for (int64_t ct = rt; ct < nw; ++ct) {
            const int64_t j = ct * kWave + lane;
            __syncthreads();
            if (j < S) {
                const int64_t g = (int64_t)a.ids[a.bmem[base + j]] * W;
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    const uint64_t xv = a.x[g + w], zv = a.z[g + w];
                    cx[lane * 2 * W + 2 * w] = (uint32_t)xv;
                    cx[lane * 2 * W + 2 * w + 1] = (uint32_t)(xv >> 32);
                    cz[lane * 2 * W + 2 * w] = (uint32_t)zv;
                    cz[lane * 2 * W + 2 * w + 1] = (uint32_t)(zv >> 32);
                }
            } else {
#pragma unroll
                for (int h = 0; h < 2 * W; ++h) cx[lane * 2 * W + h] = cz[lane * 2 * W + h] = 0u;
            }
            __syncthreads();
            uint32_t lo = 0u, hi = 0u;
#pragma unroll
            for (int jj = 0; jj < 32; ++jj) lo |= pair_bit<W, REL>(xi, zi, &cx[jj * 2 * W], &cz[jj * 2 * W]) << jj;
#pragma unroll
            for (int jj = 0; jj < 32; ++jj)
                hi |= pair_bit<W, REL>(xi, zi, &cx[(jj + 32) * 2 * W], &cz[(jj + 32) * 2 * W]) << jj;
            uint64_t row = ((uint64_t)hi << 32) | lo;
            if (i >= S) row = 0;
            if (ct == rt) {
                // keep the upper triangle (columns after the row), then add
                // its transpose: the row's bits for earlier members
                row &= lane == 63 ? 0ull : (~0ull << (lane + 1));
                const uint64_t col = wave_transpose64(row);
                if (i < S) Rm[i * nw + rt] = row | col;
            } else {
                const uint64_t col = wave_transpose64(row);
                if (i < S) Rm[i * nw + ct] = row;
                if (j < S) Rm[j * nw + rt] = col;
            }
        }
    }
}

// ---- pairs sharing a smaller colour -------------------------------------
// Member p of bucket c has prefix L(v_p)[0..k_p), the colours below c.  Two
// members share a smaller colour iff some colour occurs in both prefixes.
// An LDS hash set finds the colours that occur twice; the (colour, member)
// entries of those colours yield the pairs, whose bits are set in D.
constexpr int kDupThreads = 256;
constexpr int kDupTable = 8192;  // slots; a bucket fits when its prefixes hold <= kDupTable/2 colours
constexpr int kDupList = 1024;
constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr uint32_t kTwice = 0x80000000u;

__device__ __forceinline__ uint32_t hash_colour(uint32_t c) { return (c * 0x9E3779B1u) >> (32 - 13); }

__global__ void __launch_bounds__(kDupThreads) dup_kernel(DupArgs a)
{
    __shared__ uint32_t table[kDupTable];
    __shared__ uint32_t lcol[kDupList];
    __shared__ uint32_t lmem[kDupList];
    __shared__ int lcount;
    __shared__ int total_prefix;
    const int t = threadIdx.x;
    for (int64_t c = blockIdx.x; c < a.P; c += gridDim.x) {
        const int64_t base = a.bstart[c];
        const int64_t S = a.bstart[c + 1] - base;
        if (S < 2) continue;
        __syncthreads();
        if (t == 0) {
            total_prefix = 0;
            lcount = 0;
        }
        __syncthreads();
        int mine = 0;
        for (int64_t p = t; p < S; p += kDupThreads) mine += a.bslot[base + p];
        atomicAdd(&total_prefix, mine);
        __syncthreads();
        const int tp = total_prefix;
        if (tp == 0) continue;
        if (2 * tp > kDupTable) {  // too many prefix colours for the table: exact per-pair check later
            if (t == 0) a.slow[atomicAdd(a.n_slow, 1)] = (uint32_t)c;
            continue;
        }
        for (int s = t; s < kDupTable; s += kDupThreads) table[s] = kEmpty;
        __syncthreads();
        for (int64_t p = t; p < S; p += kDupThreads) {
            const int k = a.bslot[base + p];
            const uint32_t *L = a.lists + (int64_t)a.bmem[base + p] * a.T;
            for (int s = 0; s < k; ++s) {
                const uint32_t col = L[s];
                uint32_t h = hash_colour(col);
                while (true) {
                    const uint32_t old = atomicCAS(&table[h], kEmpty, col);
                    if (old == kEmpty) break;
                    if ((old & ~kTwice) == col) {
                        atomicOr(&table[h], kTwice);
                        break;
                    }
                    h = (h + 1) & (kDupTable - 1);
                }
            }
        }
        __syncthreads();
        bool overflow = false;
        for (int64_t p = t; p < S; p += kDupThreads) {
            const int k = a.bslot[base + p];
            const uint32_t *L = a.lists + (int64_t)a.bmem[base + p] * a.T;
            for (int s = 0; s < k; ++s) {
                const uint32_t col = L[s];
                uint32_t h = hash_colour(col);
                while ((table[h] & ~kTwice) != col) h = (h + 1) & (kDupTable - 1);
                if (table[h] & kTwice) {
                    const int e = atomicAdd(&lcount, 1);
                    if (e < kDupList) {
                        lcol[e] = col;
                        lmem[e] = (uint32_t)p;
                    } else {
                        overflow = true;
                    }
                }
            }
        }
        __syncthreads();
        const int n = lcount;
        if (n > kDupList) {
            if (t == 0) a.slow[atomicAdd(a.n_slow, 1)] = (uint32_t)c;
            continue;
        }
        (void)overflow;
        const int64_t nw = (S + 63) >> 6;
        uint64_t *Dm = a.D + a.rb_off[c];
        for (int e = t; e < n; e += kDupThreads)
            for (int f = 0; f < n; ++f)
                if (f != e && lcol[f] == lcol[e]) {
                    const uint32_t p = lmem[e], q = lmem[f];
                    atomicOr((unsigned long long *)&Dm[(int64_t)p * nw + (q >> 6)], 1ull << (q & 63));
                }
    }
}

// Buckets whose prefixes overflow the LDS table: test every pair directly by
// merging the two prefixes (rare: only very large buckets).
__global__ void __launch_bounds__(256) dup_slow_kernel(DupArgs a, int64_t n_slow)
{
    for (int64_t b = blockIdx.x; b < n_slow; b += gridDim.x) {
        const int64_t c = a.slow[b];
        const int64_t base = a.bstart[c];
        const int64_t S = a.bstart[c + 1] - base;
        const int64_t nw = (S + 63) >> 6;
        uint64_t *Dm = a.D + a.rb_off[c];
        for (int64_t p = threadIdx.x; p < S; p += blockDim.x) {
            const int kp = a.bslot[base + p];
            if (kp == 0) continue;
            const uint32_t *Lp = a.lists + (int64_t)a.bmem[base + p] * a.T;
            for (int64_t q = 0; q < S; ++q) {
                const int kq = a.bslot[base + q];
                if (q == p || kq == 0) continue;
                const uint32_t *Lq = a.lists + (int64_t)a.bmem[base + q] * a.T;
                int x = 0, y = 0;
                bool shared = false;
                while (x < kp && y < kq) {
                    if (Lp[x] == Lq[y]) {
                        shared = true;
                        break;
                    }
                    if (Lp[x] < Lq[y]) ++x;
                    else ++y;
                }
                if (shared) atomicOr((unsigned long long *)&Dm[p * nw + (q >> 6)], 1ull << (q & 63));
            }
        }
    }
}

// Conflict-edge count of every member: popcount(R & ~D) of its row, stored
// at the member's (vertex, slot) position.
__global__ void __launch_bounds__(kWave) count_kernel(CsrArgs a)
{
    for (int64_t c = blockIdx.x; c < a.P; c += gridDim.x) {
        const int64_t base = a.bstart[c];
        const int64_t S = a.bstart[c + 1] - base;
        const int64_t nw = (S + 63) >> 6;
        const uint64_t *Rm = a.R + a.rb_off[c];
        const uint64_t *Dm = a.D + a.rb_off[c];
        for (int64_t p = threadIdx.x; p < S; p += kWave) {
            int cnt = 0;
            for (int64_t w = 0; w < nw; ++w) cnt += __popcll(Rm[p * nw + w] & ~Dm[p * nw + w]);
            a.slot_cnt[(int64_t)a.bmem[base + p] * a.T + a.bslot[base + p]] = cnt;
        }
    }
}

// CSR rows: each member's edges in this bucket go to its (vertex, slot)
// segment, whose start comes from the exclusive scan of the counts.
__global__ void __launch_bounds__(kWave) fill_kernel(CsrArgs a)
{
    for (int64_t c = blockIdx.x; c < a.P; c += gridDim.x) {
        const int64_t base = a.bstart[c];
        const int64_t S = a.bstart[c + 1] - base;
        const int64_t nw = (S + 63) >> 6;
        const uint64_t *Rm = a.R + a.rb_off[c];
        const uint64_t *Dm = a.D + a.rb_off[c];
        for (int64_t p = threadIdx.x; p < S; p += kWave) {
            int64_t at = a.slot_off[(int64_t)a.bmem[base + p] * a.T + a.bslot[base + p]];
            for (int64_t w = 0; w < nw; ++w) {
                uint64_t bits = Rm[p * nw + w] & ~Dm[p * nw + w];
                while (bits) {
                    const int b = __builtin_ctzll(bits);
                    bits &= bits - 1;
                    a.adj[at++] = (int32_t)a.bmem[base + w * 64 + b];
                }
            }
        }
    }
}

__global__ void rowptr_kernel(const int64_t *slot_off, int64_t m, int32_t T, int64_t *rowptr)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v <= m; v += (int64_t)gridDim.x * blockDim.x)
        rowptr[v] = slot_off[v * T];
}

unsigned grid_cap(int64_t items, int64_t cap = 1 << 22)
{
    if (items < 1) items = 1;
    return (unsigned)(items < cap ? items : cap);
}

}  // namespace

void launch_relate(const RelateArgs &a, hipStream_t st)
{
    if (a.total_row_tiles <= 0) return;
    const unsigned grid = grid_cap(a.total_row_tiles);
#define PICASSO_REL_CASE(WW)                                                                       \
    case WW:                                                                                       \
        if (a.relation == PICASSO_REL_ANTICOMMUTE)                                                 \
            relate_kernel<WW, PICASSO_REL_ANTICOMMUTE><<<grid, kWave, 0, st>>>(a);                 \
        else                                                                                       \
            relate_kernel<WW, PICASSO_REL_QWC><<<grid, kWave, 0, st>>>(a);                         \
        break;
    switch (a.W) {
        PICASSO_REL_CASE(1)
        PICASSO_REL_CASE(2)
        PICASSO_REL_CASE(3)
        PICASSO_REL_CASE(4)
        default:
            throw Error(PICASSO_EINTERNAL, "relate kernel: unsupported word count");
    }
#undef PICASSO_REL_CASE
    PCHECK_LAUNCH();
}

void launch_dup(const DupArgs &a, hipStream_t st)
{
    if (a.P <= 0) return;
    dup_kernel<<<grid_cap(a.P, 1 << 20), kDupThreads, 0, st>>>(a);
    PCHECK_LAUNCH();
}

void launch_dup_slow(const DupArgs &a, int64_t n_slow, hipStream_t st)
{
    if (n_slow <= 0) return;
    dup_slow_kernel<<<grid_cap(n_slow, 1 << 16), 256, 0, st>>>(a, n_slow);
    PCHECK_LAUNCH();
}

void launch_count(const CsrArgs &a, hipStream_t st)
{
    if (a.P <= 0) return;
    count_kernel<<<grid_cap(a.P, 1 << 20), kWave, 0, st>>>(a);
    PCHECK_LAUNCH();
}

void launch_fill(const CsrArgs &a, hipStream_t st)
{
    if (a.P <= 0) return;
    fill_kernel<<<grid_cap(a.P, 1 << 20), kWave, 0, st>>>(a);
    PCHECK_LAUNCH();
}

void launch_rowptr(const int64_t *slot_off, int64_t m, int32_t T, int64_t *rowptr, hipStream_t st)
{
    const int64_t b = (m + 1 + 255) / 256;
    rowptr_kernel<<<grid_cap(b, 65535 * 16), 256, 0, st>>>(slot_off, m, T, rowptr);
    PCHECK_LAUNCH();
}

}  // namespace picasso
