// Intra-bucket pair kernels: the conflict-graph build (Alg. 1
// construct_conflict_graph; Sec. IV-A; the CSR output of Alg. 3).
//
// A pair {u, v} conflicts iff the relation holds and L(u), L(v) share a
// colour.  Such a pair lies in the bucket of each shared colour; it is kept
// once, in the bucket of its smallest shared colour c.  Lists are sorted, so
// "no smaller shared colour" means the list prefixes before c are disjoint.
//
// Per bucket two S x S bit matrices sit in HBM, row p holding ceil(S/64)
// words:
//   R: relation bits between members (symmetric; relate.hip);
//   D: pairs that share a colour smaller than the bucket's (dup_kernel).
// The bucket's conflict edges are R & ~D (D is read only for the members
// whose dflag byte says their row has a bit).  count_kernel pop-counts each
// row into the member's (vertex, slot) segment length; per-vertex prefixes
// and a scan of the row lengths place the segments, and fill_kernel expands
// each row into its CSR segment.  The colouring reads
// the lower triangle of R (earlier members) directly.
#include "common.h"

namespace picasso {
namespace {

constexpr int kWave = 64;

// ---- pairs sharing a smaller colour -------------------------------------
// Member p of bucket c has prefix L(v_p)[0..k_p), the colours below c.  Two
// members share a smaller colour iff some colour occurs in both prefixes.
// When the instance's colours below c span at most kDupSpan, each member's
// prefix becomes a bitset over that span and D's rows are written whole from
// pairwise intersections.  Otherwise, a pass over the bucket's prefix entries marks each colour in two LDS
// bitmaps (seen once, seen again); a second pass lists the entries whose
// bit was seen again, as (colour, member); every two members listed with one
// colour get their bit set in D (lists of up to kDupScan entries by comparing
// each entry with the later ones, longer ones by sorting and pairing runs).
//  - First attempt: one pass over all entries, bits indexed by a
//    multiplicative hash of the colour.  Two colours sharing a bit only add
//    entries to the list (runs are taken on the colour itself).  Each
//    thread keeps the entries it fetched in registers for the second pass.
//  - If that list overflows (narrow palettes, where most prefix colours are
//    shared), exact windows of colours below c, halved until the list fits;
//    below 64 colours the bucket takes the exact per-pair check.
// Each member's list start is staged in LDS with the prefix-length scan, so
// an entry costs one load (entry e -> member by a search of the scan).
constexpr int kDupThreads = 256;
constexpr int kDupHashBits = 15;                 // hashed bitmap: 2^15 bits
constexpr int kDupBits = 1 << 15;                // bits per bitmap (window of colours)
constexpr int kDupWords = kDupBits / 32;
constexpr int kDupMembers = 1024;                // larger buckets take the exact per-pair check
constexpr int kDupList = 2048;                   // listed entries (power of two)
constexpr int kDupHeld = 16;                     // entries a thread keeps between the passes
constexpr int kDupScan = 512;                    // lists up to this long are paired by hash groups (fit the seen bitmap)
constexpr int kDupSpan = 512;                    // colour ranges up to this wide use member bitsets
constexpr int kDupBatch = 8;
constexpr uint32_t kNone = 0xFFFFFFFFu;
// pair_scan reuses the two bitmaps: `seen` holds up to kDupScan listed
// entries, `again` 256 counts and 257 offsets
static_assert(kDupScan * sizeof(uint64_t) <= kDupWords * sizeof(uint32_t), "pair_scan's entries must fit `seen`");
static_assert(256 + 257 <= kDupWords, "pair_scan's counts and offsets must fit `again`");
static_assert(kDupScan <= kDupList && (kDupList & (kDupList - 1)) == 0, "list sizes");

__device__ __forceinline__ uint32_t dup_hash(uint32_t colour)
{
    return (colour * 0x9E3779B1u) >> (32 - kDupHashBits);
}

__global__ void __launch_bounds__(kDupThreads) dup_kernel(DupArgs a)
{
    __shared__ uint32_t seen[kDupWords], again[kDupWords];
    __shared__ int64_t lbase[kDupMembers];  // first list entry of each member's vertex
    __shared__ int32_t koff[kDupMembers + 1];
    __shared__ uint64_t list[kDupList];     // colour << 32 | member
    __shared__ int wsum[kDupThreads / 64];
    __shared__ int lcount;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    for (int64_t c = blockIdx.x; c < a.P; c += gridDim.x) {
        const int64_t base = a.bstart[c];
        const int S = (int)(a.bstart[c + 1] - base);
        if (S < 2) continue;
        if (S > kDupMembers) {
            if (t == 0) a.slow[atomicAdd(a.n_slow, 1)] = (uint32_t)c;
            continue;
        }
        // member list starts and the exclusive scan of their prefix lengths
        __syncthreads();
        int chunk_base = 0;
        for (int p0 = 0; p0 < S; p0 += kDupThreads) {
            const int p = p0 + t;
            int k = 0;
            if (p < S) {
                lbase[p] = a.bent[base + p] - a.bslot[base + p];
                k = a.bslot[base + p];
            }
            int inc = k;
            for (int d = 1; d < 64; d <<= 1) {
                const int o = __shfl_up(inc, d, 64);
                if (lane >= d) inc += o;
            }
            if (lane == 63) wsum[wave] = inc;
            __syncthreads();
            int before = chunk_base;
            int all = 0;
            for (int w = 0; w < kDupThreads / 64; ++w) {
                if (w < wave) before += wsum[w];
                all += wsum[w];
            }
            if (p < S) koff[p] = before + inc - k;
            chunk_base += all;
            __syncthreads();
        }
        const int total = chunk_base;
        if (total < 2) continue;
        if (t == 0) koff[S] = total;
        const int64_t nw = (S + 63) >> 6;
        uint64_t *Dm = a.D + a.rb_off[c];
        auto set_pair = [&](uint32_t pe, uint32_t pf) {
            atomicOr((unsigned long long *)&Dm[(int64_t)pe * nw + (pf >> 6)], 1ull << (pf & 63));
            atomicOr((unsigned long long *)&Dm[(int64_t)pf * nw + (pe >> 6)], 1ull << (pe & 63));
            a.dflag[base + pe] = 1;
            a.dflag[base + pf] = 1;
        };
        auto fetch = [&](int e, uint32_t &col, int &mem) {
            int l = 0, h = S;  // koff[l] <= e < koff[h]
            while (h - l > 1) {
                const int mid = (l + h) >> 1;
                if (koff[mid] <= e) l = mid;
                else h = mid;
            }
            mem = l;
            col = a.lists[lbase[l] + (e - koff[l])];
        };
        auto mark = [&](uint32_t b) {
            const uint32_t bit = 1u << (b & 31);
            if (atomicOr(&seen[b >> 5], bit) & bit) atomicOr(&again[b >> 5], bit);
        };
        auto enlist = [&](uint32_t b, uint32_t cc, int mem) {
            if (again[b >> 5] & (1u << (b & 31))) {
                const int at = atomicAdd(&lcount, 1);
                if (at < kDupList) list[at] = ((uint64_t)cc << 32) | (uint32_t)mem;
            }
        };
        auto clear = [&](int words) {
            __syncthreads();
            for (int w = t; w < words; w += kDupThreads) seen[w] = again[w] = 0u;
            if (t == 0) lcount = 0;
            __syncthreads();
        };
        // sorts the list (n entries) by (colour, member)
        auto sort_list = [&](int n) {
            int N = 2;
            while (N < n) N <<= 1;
            for (int e = n + t; e < N; e += kDupThreads) list[e] = ~0ull;
            __syncthreads();
            for (int k = 2; k <= N; k <<= 1)
                for (int j = k >> 1; j > 0; j >>= 1) {
                    for (int e = t; e < N; e += kDupThreads) {
                        const int f = e ^ j;
                        if (f > e) {
                            const uint64_t ve = list[e], vf = list[f];
                            if ((ve > vf) == ((e & k) == 0)) {
                                list[e] = vf;
                                list[f] = ve;
                            }
                        }
                    }
                    __syncthreads();
                }
        };
        // lists of up to kDupScan entries: a counting sort by an 8-bit hash of
        // the colour into the (then free) bitmap space, and every two entries
        // of one colour paired inside their hash group by one thread
        auto pair_scan = [&](int n) {
            uint32_t *hcnt = again;                                        // 256 counts
            uint32_t *hoff = again + 256;                                  // 257 offsets
            uint64_t *grp = reinterpret_cast<uint64_t *>(seen);            // n entries by group
            __syncthreads();
            for (int g = t; g < 256; g += kDupThreads) hcnt[g] = 0u;
            __syncthreads();
            for (int e = t; e < n; e += kDupThreads) atomicAdd(&hcnt[dup_hash((uint32_t)(list[e] >> 32)) & 255u], 1u);
            __syncthreads();
            if (t < 64) {  // exclusive scan of the 256 counts, one wave, 4 per lane
                uint32_t v[4], sum = 0u;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    v[k] = hcnt[t * 4 + k];
                    sum += v[k];
                }
                uint32_t inc = sum;
                for (int d = 1; d < 64; d <<= 1) {
                    const uint32_t o = __shfl_up(inc, d, 64);
                    if (t >= d) inc += o;
                }
                uint32_t run = inc - sum;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    hoff[t * 4 + k] = run;
                    run += v[k];
                }
                if (t == 63) hoff[256] = inc;
            }
            __syncthreads();
            for (int g = t; g < 256; g += kDupThreads) hcnt[g] = hoff[g];  // fill cursors
            __syncthreads();
            for (int e = t; e < n; e += kDupThreads) {
                const uint64_t le = list[e];
                grp[atomicAdd(&hcnt[dup_hash((uint32_t)(le >> 32)) & 255u], 1u)] = le;
            }
            __syncthreads();
            for (int g = t; g < 256; g += kDupThreads)
                for (uint32_t e = hoff[g]; e < hoff[g + 1]; ++e) {
                    const uint32_t ce = (uint32_t)(grp[e] >> 32), pe = (uint32_t)grp[e];
                    for (uint32_t f = e + 1; f < hoff[g + 1]; ++f)
                        if ((uint32_t)(grp[f] >> 32) == ce) set_pair(pe, (uint32_t)grp[f]);
                }
        };
        // each listed entry of a sorted list pairs with the later entries of its colour run
        auto pair_runs = [&](int n) {
            for (int e = t; e < n; e += kDupThreads) {
                const uint32_t ce = (uint32_t)(list[e] >> 32), pe = (uint32_t)list[e];
                for (int f = e + 1; f < n && (uint32_t)(list[f] >> 32) == ce; ++f) set_pair(pe, (uint32_t)list[f]);
            }
        };
        // narrow colour range below c: each member's prefix as a bitset over
        // it, and D's rows written whole as "bitsets intersect" (pairs sharing
        // a colour are then common, too many to list one by one)
        const int64_t pal = a.inst[a.binst[c]].pal;
        const int sw = (int)((c - pal + 63) >> 6);  // bitset words per member
        if (c - pal <= kDupSpan && (int64_t)S * sw <= kDupList) {
            uint64_t *bits = list;  // S x sw words
            __syncthreads();
            for (int p = t; p < S; p += kDupThreads) {
                uint64_t b[kDupSpan / 64];
#pragma unroll
                for (int w = 0; w < kDupSpan / 64; ++w) b[w] = 0ull;
                const int k = koff[p + 1] - koff[p];
                for (int i = 0; i < k; ++i) {
                    const uint32_t cc = a.lists[lbase[p] + i] - (uint32_t)pal;
#pragma unroll
                    for (int w = 0; w < kDupSpan / 64; ++w)
                        if ((int)(cc >> 6) == w) b[w] |= 1ull << (cc & 63);
                }
                for (int w = 0; w < sw; ++w) bits[p * sw + w] = b[w];
            }
            __syncthreads();
            for (int64_t x = t; x < (int64_t)S * nw; x += kDupThreads) {
                const int p = (int)(x / nw), w = (int)(x - (int64_t)p * nw);
                uint64_t row = 0ull;
                for (int b = 0; b < 64; ++b) {
                    const int q = w * 64 + b;
                    if (q >= S || q == p) continue;
                    uint64_t any = 0ull;
                    for (int u = 0; u < sw; ++u) any |= bits[p * sw + u] & bits[q * sw + u];
                    if (any) row |= 1ull << b;
                }
                Dm[x] = row;
                if (row) a.dflag[base + p] = 1;
            }
            continue;
        }
        // first attempt: hashed bits over all entries (held in registers
        // between the passes when they fit, fetched twice otherwise)
        clear(kDupWords);
        if (total <= kDupThreads * kDupHeld) {
            uint32_t col[kDupHeld];
            int mem[kDupHeld];
#pragma unroll
            for (int j = 0; j < kDupHeld; ++j) {
                const int e = t + j * kDupThreads;
                col[j] = kNone;
                mem[j] = 0;
                if (e < total) fetch(e, col[j], mem[j]);
            }
#pragma unroll
            for (int j = 0; j < kDupHeld; ++j)
                if (col[j] != kNone) mark(dup_hash(col[j]));
            __syncthreads();
#pragma unroll
            for (int j = 0; j < kDupHeld; ++j)
                if (col[j] != kNone) enlist(dup_hash(col[j]), col[j], mem[j]);
        } else {
            for (int round = 0; round < 2; ++round) {  // 0: mark, 1: list colours seen again
                for (int e0 = t; e0 < total; e0 += kDupThreads * kDupBatch) {
                    uint32_t col[kDupBatch];
                    int mem[kDupBatch];
#pragma unroll
                    for (int j = 0; j < kDupBatch; ++j) {
                        const int e = e0 + j * kDupThreads;
                        col[j] = kNone;
                        mem[j] = 0;
                        if (e < total) fetch(e, col[j], mem[j]);
                    }
#pragma unroll
                    for (int j = 0; j < kDupBatch; ++j) {
                        if (col[j] == kNone) continue;
                        if (round == 0) mark(dup_hash(col[j]));
                        else enlist(dup_hash(col[j]), col[j], mem[j]);
                    }
                }
                if (round == 0) __syncthreads();
            }
        }
        __syncthreads();
        const int n0 = lcount;
        if (n0 <= kDupList) {
            if (n0 > kDupScan) {
                sort_list(n0);
                pair_runs(n0);
            } else if (n0 >= 2) {
                pair_scan(n0);
            }
            continue;
        }
        // exact windows of colours below c
        bool overflow = false;
        int64_t lo = pal, win = kDupBits;  // colours below c of this instance
        while (lo < c) {
            const int64_t hi = lo + win < c ? lo + win : c;
            clear((int)((hi - lo + 31) >> 5));
            for (int round = 0; round < 2; ++round) {  // 0: mark, 1: list colours seen again
                for (int e0 = t; e0 < total; e0 += kDupThreads * kDupBatch) {
                    uint32_t col[kDupBatch];
                    int mem[kDupBatch];
#pragma unroll
                    for (int j = 0; j < kDupBatch; ++j) {
                        const int e = e0 + j * kDupThreads;
                        col[j] = kNone;
                        mem[j] = 0;
                        if (e < total) fetch(e, col[j], mem[j]);
                    }
#pragma unroll
                    for (int j = 0; j < kDupBatch; ++j) {
                        const uint32_t cc = col[j];
                        if (cc == kNone || cc < lo || cc >= hi) continue;
                        if (round == 0) mark(cc - (uint32_t)lo);
                        else enlist(cc - (uint32_t)lo, cc, mem[j]);
                    }
                }
                __syncthreads();
            }
            const int n = lcount;
            if (n > kDupList) {  // narrower window
                if (win <= 64) {
                    overflow = true;
                    break;
                }
                win >>= 1;
                continue;
            }
            if (n > kDupScan) {
                sort_list(n);
                pair_runs(n);
            } else if (n >= 2) {
                pair_scan(n);
            }
            lo = hi;
        }
        if (overflow && t == 0) a.slow[atomicAdd(a.n_slow, 1)] = (uint32_t)c;
    }
}

// Buckets the LDS pass cannot take: every relation pair is checked directly
// by merging the two prefixes (rare: only very large buckets).
__global__ void __launch_bounds__(256) dup_slow_kernel(DupArgs a)
{
    const int64_t n_slow = *a.n_slow;
    for (int64_t b = blockIdx.x; b < n_slow; b += gridDim.x) {
        const int64_t c = a.slow[b];
        const int64_t base = a.bstart[c];
        const int64_t S = a.bstart[c + 1] - base;
        const int64_t nw = (S + 63) >> 6;
        const uint64_t *Rm = a.R + a.rb_off[c];
        uint64_t *Dm = a.D + a.rb_off[c];
        for (int64_t p = threadIdx.x; p < S; p += blockDim.x) {
            const int kp = a.bslot[base + p];
            if (kp == 0) continue;
            const uint32_t *Lp = a.lists + (a.bent[base + p] - a.bslot[base + p]);
            for (int64_t w = 0; w < nw; ++w) {
                uint64_t bits = Rm[p * nw + w];
                while (bits) {
                    const int64_t q = w * 64 + __builtin_ctzll(bits);
                    bits &= bits - 1;
                    const int kq = a.bslot[base + q];
                    if (kq == 0) continue;
                    const uint32_t *Lq = a.lists + (a.bent[base + q] - a.bslot[base + q]);
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
                    if (shared) {
                        atomicOr((unsigned long long *)&Dm[p * nw + (q >> 6)], 1ull << (q & 63));
                        a.dflag[base + p] = 1;
                    }
                }
            }
        }
    }
}

// Conflict-edge count of every member: popcount(R & ~D) of its row, stored
// at the member's (vertex, slot) segment.  Buckets of up to kCountMembers
// members are read word by word across the lanes (consecutive lanes,
// consecutive words of the bucket's block), each row's popcounts summed in
// LDS; larger buckets take one thread per row.
constexpr int kCountThreads = 256;
constexpr int kCountMembers = 1024;

__global__ void __launch_bounds__(kCountThreads) count_kernel(CsrArgs a)
{
    __shared__ int cnt[kCountMembers];
    const int t = threadIdx.x;
    for (int64_t c = blockIdx.x; c < a.P; c += gridDim.x) {
        const int64_t base = a.bstart[c];
        const int64_t S = a.bstart[c + 1] - base;
        const int64_t nw = (S + 63) >> 6;
        const uint64_t *Rm = a.R + a.rb_off[c];
        const uint64_t *Dm = a.D + a.rb_off[c];
        if (S <= kCountMembers) {
            __syncthreads();
            for (int p = t; p < (int)S; p += kCountThreads) cnt[p] = 0;
            __syncthreads();
            const int words = (int)(S * nw), nw32 = (int)nw;
            for (int x = t; x < words; x += kCountThreads) {
                const int p = x / nw32;
                uint64_t r = Rm[x];
                if (a.dflag[base + p]) r &= ~Dm[x];
                const int k = __popcll(r);
                if (k) atomicAdd(&cnt[p], k);
            }
            __syncthreads();
            for (int p = t; p < (int)S; p += kCountThreads)
                a.seg[(int64_t)a.bslot[base + p] * a.seg_m + a.bmem[base + p]] = cnt[p];
        } else {
            for (int64_t p = t; p < S; p += kCountThreads) {
                int k = 0;
                if (a.dflag[base + p]) {
                    for (int64_t w = 0; w < nw; ++w) k += __popcll(Rm[p * nw + w] & ~Dm[p * nw + w]);
                } else {
                    for (int64_t w = 0; w < nw; ++w) k += __popcll(Rm[p * nw + w]);
                }
                a.seg[(int64_t)a.bslot[base + p] * a.seg_m + a.bmem[base + p]] = k;
            }
        }
    }
}

// CSR rows: one wave per member row.  The 64 lanes test the 64 bits of a
// row word, and a ballot prefix count (mbcnt) gives each set bit its slot in
// the member's contiguous (vertex, slot) segment, so every store of the
// wave lands in one run of the CSR.  When the bucket fits the stage, its
// rows of R & ~D, member ids and segment offsets are first staged in LDS
// with independent loads.  The stage is sized by the launch to the largest
// bucket (capped), so that small buckets leave room for many workgroups per
// CU: the staging loads are a chain of dependent reads whose latency only
// other resident workgroups hide.
constexpr int kFillWaves = 4;
constexpr int64_t kFillMembers = 1024;
constexpr int64_t kFillWords = 4096;

__global__ void __launch_bounds__(kWave * kFillWaves) fill_kernel(CsrArgs a, int64_t cap_members, int64_t cap_words)
{
    extern __shared__ uint64_t fill_lds[];
    uint64_t *rows = fill_lds;                                         // cap_words
    int64_t *seg = reinterpret_cast<int64_t *>(fill_lds + cap_words); // cap_members
    uint32_t *mv = reinterpret_cast<uint32_t *>(seg + cap_members);    // cap_members
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (a.skip && *a.skip) return;  // the CSR does not fit the buffer: nothing is written
    for (int64_t c = blockIdx.x; c < a.P; c += gridDim.x) {
        const int64_t base = a.bstart[c];
        const int64_t S = a.bstart[c + 1] - base;
        if (S < 2) continue;
        const int64_t nw = (S + 63) >> 6;
        const uint64_t *Rm = a.R + a.rb_off[c];
        const uint64_t *Dm = a.D + a.rb_off[c];
        if (S <= cap_members && S * nw <= cap_words) {
            __syncthreads();
            for (int64_t p = threadIdx.x; p < S; p += blockDim.x) {
                const uint32_t v = a.bmem[base + p];
                mv[p] = v;
                seg[p] = a.seg_off[(int64_t)a.bslot[base + p] * a.seg_m + v];
            }
            // D is read only for the rows that have a bit in it
            for (int64_t w = threadIdx.x; w < S * nw; w += blockDim.x) {
                const uint64_t r = Rm[w];
                rows[w] = a.dflag[base + w / nw] ? r & ~Dm[w] : r;
            }
            __syncthreads();
            for (int64_t p = wave; p < S; p += kFillWaves) {
                if ((int64_t)mv[p] < a.v_lo || (int64_t)mv[p] >= a.v_hi) continue;  // another chunk's row
                int64_t at = seg[p] - a.adj_base;
                for (int64_t w = 0; w < nw; ++w) {
                    const uint64_t bits = rows[p * nw + w];
                    const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(bits >> 32),
                                                               __builtin_amdgcn_mbcnt_lo((uint32_t)bits, 0u));
                    if ((bits >> lane) & 1ull) a.adj[at + rank] = (int32_t)mv[w * 64 + lane];
                    at += __popcll(bits);
                }
            }
        } else {
            for (int64_t p = wave; p < S; p += kFillWaves) {
                const int64_t v = a.bmem[base + p];
                if (v < a.v_lo || v >= a.v_hi) continue;  // another chunk's row
                int64_t at = a.seg_off[(int64_t)a.bslot[base + p] * a.seg_m + v] - a.adj_base;
                const bool dd = a.dflag[base + p];
                for (int64_t w = 0; w < nw; ++w) {
                    const uint64_t bits = dd ? Rm[p * nw + w] & ~Dm[p * nw + w] : Rm[p * nw + w];
                    const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(bits >> 32),
                                                               __builtin_amdgcn_mbcnt_lo((uint32_t)bits, 0u));
                    if ((bits >> lane) & 1ull) a.adj[at + rank] = (int32_t)a.bmem[base + w * 64 + lane];
                    at += __popcll(bits);
                }
            }
        }
    }
}

// One thread per vertex; for each slot the threads of a wave touch
// consecutive vertices of one slot row.
__global__ void row_lengths_kernel(const int32_t *seg, int64_t m, const int64_t *loff, int32_t *deg)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < m; v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t T = loff[v + 1] - loff[v];
        int32_t run = 0;
        for (int64_t s = 0; s < T; ++s) run += seg[s * m + v];
        deg[v] = run;
    }
}

__global__ void seg_offsets_kernel(const int32_t *seg, int64_t m, const int64_t *loff, const int64_t *rowptr,
                                   int64_t *seg_off)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < m; v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t T = loff[v + 1] - loff[v];
        int64_t at = rowptr[v];
        for (int64_t s = 0; s < T; ++s) {
            seg_off[s * m + v] = at;
            at += seg[s * m + v];
        }
    }
}

unsigned grid_cap(int64_t items, int64_t cap = 1 << 22)
{
    if (items < 1) items = 1;
    return (unsigned)(items < cap ? items : cap);
}

}  // namespace

void launch_dup(const DupArgs &a, hipStream_t st)
{
    if (a.P <= 0) return;
    dup_kernel<<<grid_cap(a.P, 1 << 20), kDupThreads, 0, st>>>(a);
    PCHECK_LAUNCH();
}

void launch_dup_slow(const DupArgs &a, hipStream_t st)
{
    if (a.P <= 0) return;
    // a fixed grid; blocks past the device-side count of slow buckets exit
    dup_slow_kernel<<<grid_cap(a.P, 1024), 256, 0, st>>>(a);
    PCHECK_LAUNCH();
}

void launch_count(const CsrArgs &a, hipStream_t st)
{
    if (a.P <= 0) return;
    count_kernel<<<grid_cap(a.P, 1 << 20), kCountThreads, 0, st>>>(a);
    PCHECK_LAUNCH();
}

void launch_fill(const CsrArgs &a, int64_t max_size, hipStream_t st)
{
    if (a.P <= 0) return;
    // stage: every bucket up to the largest one present, within the caps
    // (larger buckets read their rows from global memory directly)
    const int64_t cap_members = std::min<int64_t>(std::max<int64_t>(max_size, 64), kFillMembers);
    const int64_t cap_words = std::min<int64_t>(cap_members * ((cap_members + 63) >> 6), kFillWords);
    const size_t lds = (size_t)cap_words * 8 + (size_t)cap_members * 12;
    fill_kernel<<<grid_cap(a.P, 1 << 20), kWave * kFillWaves, lds, st>>>(a, cap_members, cap_words);
    PCHECK_LAUNCH();
}

__global__ void csr_guard_kernel(const int64_t *total, int64_t cap, int32_t *flag) { *flag = *total > cap; }

void launch_csr_guard(const int64_t *total, int64_t cap, int32_t *flag, hipStream_t st)
{
    csr_guard_kernel<<<1, 1, 0, st>>>(total, cap, flag);
    PCHECK_LAUNCH();
}

void launch_row_lengths(const int32_t *seg, int64_t m, const int64_t *loff, int32_t *deg, hipStream_t st)
{
    if (m <= 0) return;
    row_lengths_kernel<<<grid_cap((m + 255) / 256, 65535 * 16), 256, 0, st>>>(seg, m, loff, deg);
    PCHECK_LAUNCH();
}

void launch_seg_offsets(const int32_t *seg, int64_t m, const int64_t *loff, const int64_t *rowptr, int64_t *seg_off,
                        hipStream_t st)
{
    if (m <= 0) return;
    seg_offsets_kernel<<<grid_cap((m + 255) / 256, 65535 * 16), 256, 0, st>>>(seg, m, loff, rowptr, seg_off);
    PCHECK_LAUNCH();
}

}  // namespace picasso
