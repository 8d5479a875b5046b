// List colouring of the conflict graph in a random static order (Sec. IV-B,
// static order schemes; Alg. 1 colour step), evaluated in parallel.
//
// Sequential rule: vertices in ascending (priority, index) order; each takes
// the smallest colour of its list that no earlier neighbour holds, or stays
// uncoloured.  An earlier neighbour u can only take a colour c from v's
// list if c is in L(u) too, i.e. u and v meet in the bucket of c.  So the
// fate of v's slot k (colour c = L(v)[k]) is decided inside bucket c alone:
//   blocked  -- an earlier relation-neighbour in bucket c took c;
//   free     -- every earlier relation-neighbour in bucket c is known not to
//               take c.
// v takes the colour of its first free slot once all smaller slots are
// blocked, and fails when every slot is blocked.  Buckets are sorted by
// priority, so "earlier" is the lower triangle of the bucket's relation
// matrix.  This is Jones-Plassmann with decisions made per list slot: a
// vertex need not wait for earlier neighbours that cannot affect its
// choice, which cuts the number of rounds from the longest monotone path of
// the conflict graph to a few tens, and the result is the sequential one.
//
// A wave resolves its bucket's members in repeated passes until nothing
// changes, publishing blocked/free slots and colours in per-vertex words that
// other buckets read.  Rounds visit only the buckets that a state change may
// have unblocked (a worklist).
#include <algorithm>

#include "common.h"


namespace picasso {
namespace {

constexpr int kWave = 64;
constexpr uint8_t ST_UNKNOWN = 0, ST_TAKEN = 1, ST_NOT = 2;

__device__ __forceinline__ uint64_t load_u64(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Put bucket c2 on the next round's worklist unless it is already waiting,
// noting the bucket position pos of the member whose state changed (members
// before it cannot change because of it, so the next sweep of c2 starts at
// its chunk).  The wave first waits for its own outstanding memory
// operations, so the state change that causes the wake is complete (state is
// written with coherent stores and atomics) before the bucket can be taken
// off a list.  No cache flush or invalidate is needed: readers use coherent
// loads.
// Bucket c2 onto the next list: its segment's counter (row `cnt` of the
// round's counters) gives its place.
__device__ __forceinline__ void append(const JpArgs &a, int64_t c2, int32_t *out, int32_t *cnt)
{
    const int64_t sg = c2 % kJpSeg;
    const int32_t at = atomicAdd(&cnt[sg * kJpCntStride], 1);
    out[sg * a.wl_cap + at] = (int32_t)c2;
}

// A bucket's wake_at word is its state on the worklists: kIdle (not listed),
// a bucket position (listed, to be swept from that position), or kBusy (being
// swept, nothing new yet).  One atomicMin both records a position and tells
// the waker whether the bucket was idle, and so is not on any list: then the
// waker lists it.  A bucket is listed once: by the waker that finds it idle,
// or by its own visitor when a position arrived while it was busy.
constexpr unsigned long long kIdle = ~0ull;
constexpr unsigned long long kBusy = ~0ull - 1ull;

__device__ __forceinline__ void wake(const JpArgs &a, int64_t c2, int64_t pos, int32_t *out, int32_t *out_count)
{
    __builtin_amdgcn_s_waitcnt(0);  // the state change is complete before its position is published
    if (atomicMin(&a.wake_at[c2], (unsigned long long)pos) == kIdle) append(a, c2, out, out_count);
}

// The blocked slots of a vertex now run up to its slot at list entry e: that
// member's bucket may let it take its colour.  Its ready byte is set first
// (a sweep reads it with the bucket's status bytes instead of the vertex's
// slot masks), then the bucket is woken at its position.
__device__ __forceinline__ void ready_and_wake(const JpArgs &a, int64_t e, int32_t *out, int32_t *out_count)
{
    const int64_t pos = a.pos_of[e];
    const uint32_t c2 = a.lists[e];
    __hip_atomic_store(&a.rdy[pos], (uint8_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    wake(a, c2, pos, out, out_count);
}

// Slot k of v (list entries from l0, T of them) was found free: v takes
// colour L(v)[k] or an earlier one, never a later one.  Every later slot
// still unknown in its bucket is marked not-taken there and its bucket is
// woken (members after v in it may have waited on v).  Groups of 4 slots:
// independent loads, one wait so the marks are complete before any wake,
// independent wakes.
__device__ __forceinline__ void release_later_slots(const JpArgs &a, int64_t l0, int k, int T, int32_t *out,
                                                    int32_t *out_count)
{
    // (slots k+1 .. T-1; the caller may pass an earlier end)
    constexpr int G = 4;
    for (int k0 = k + 1; k0 < T; k0 += G) {
        int64_t pos[G];
        uint32_t cc[G];
        bool need[G];
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const bool ok = k0 + j < T;
            pos[j] = ok ? a.pos_of[l0 + k0 + j] : 0;
            cc[j] = ok ? a.lists[l0 + k0 + j] : 0u;
            need[j] = ok;
        }
#pragma unroll
        for (int j = 0; j < G; ++j)
            if (need[j]) need[j] = __hip_atomic_load(&a.st[pos[j]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                                   ST_UNKNOWN;
#pragma unroll
        for (int j = 0; j < G; ++j)
            if (need[j]) __hip_atomic_store(&a.st[pos[j]], ST_NOT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_s_waitcnt(0);  // the marks are complete before their positions are published
        unsigned long long old[G];
#pragma unroll
        for (int j = 0; j < G; ++j) old[j] = need[j] ? atomicMin(&a.wake_at[cc[j]], (unsigned long long)pos[j]) : 0ull;
#pragma unroll
        for (int j = 0; j < G; ++j)
            if (old[j] == kIdle) append(a, cc[j], out, out_count);
    }
}

// First slot of v not known blocked (T if all are).
__device__ __forceinline__ int first_open(const uint64_t *blk, int T)
{
    for (int w = 0; w * 64 < T; ++w) {
        const uint64_t free_bits = ~load_u64(&blk[w]);
        if (free_bits) {
            const int k = w * 64 + __builtin_ctzll(free_bits);
            return k < T ? k : T;
        }
    }
    return T;
}

constexpr int kJpStage = 1024;  // members whose (vertex, slot) are staged in LDS
static_assert(kJpSeg == kWave, "a round's workgroup (one wave) scans the segment lengths lane by lane");
constexpr int kJpResweeps = 4;  // extra sweeps of a bucket woken again during its sweep

// Resolve what can be resolved in bucket c.  A member depends only on the
// members before it in the bucket's priority order (a vertex appears in a
// bucket once), so one sweep in that order reaches the fixpoint: the wave
// walks the bucket in chunks of 64 members, each lane testing its member's
// relation row prefix against the chunk states (taken / unknown bits in LDS);
// dependencies inside a chunk settle in registers (ballots), and the chunk's
// final taken/unknown bits are what later chunks see.  Whether v's lower
// slots are all blocked is read from the member's ready byte (set by the
// wave that blocked the last of them), beside its status byte, and the
// chunk's decisions are published after the settle, so the settle steps wait
// on no memory and no sweep reads per-vertex words at scattered addresses.
// What other buckets
// decide about v reaches this bucket through the status bytes: a slot found
// free marks v's later slots not-taken there, and v's earlier slots are
// blocked, so a vertex coloured elsewhere never looks undecided here for long
// (and any step taken on it meanwhile is harmless: blocking a slot of a
// coloured vertex, or finding a slot free that it will not take).
// Cross-bucket effects wake the buckets they may unblock:
//  - a slot of v found free for the first time: v will not take any later
//    slot, so v's later slots still unknown are marked not-taken and their
//    buckets woken;
//  - a blocked slot that completes v's blocked prefix up to slot f: the
//    bucket of f is woken (v may now take it).
// Taking a colour needs no wake of its own: the slot was found free first.
__device__ void resolve_bucket(const JpArgs &a, int64_t c, uint64_t from, uint64_t *tak, uint64_t *unk,
                               uint32_t *mv, slot_t *mk, int32_t *out, int32_t *out_count)
{
    const int lane = threadIdx.x;
    const int64_t base = a.bstart[c];
    const int64_t S = a.bstart[c + 1] - base;
    const int64_t nw = (S + 63) >> 6;
    const uint64_t *Rm = a.R + a.rb_off[c];
    const bool staged = S <= kJpStage;
    // the bucket's members share an instance: list size and list offsets from its record
    const InstRec &ir = a.inst[a.binst[c]];
    const int T = ir.T;
    // the bucket's taken/unknown words, one ballot per chunk of 64 members
    __syncthreads();
    for (int64_t w = 0; w < nw; ++w) {
        const int64_t p = w * kWave + lane;
        uint8_t s = ST_NOT;
        if (p < S) {
            // coherent load: a re-sweep in the same launch must see other
            // workgroups' marks, which may sit in another XCD's cache otherwise
            s = __hip_atomic_load(&a.st[base + p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (staged) {
                mv[p] = a.bmem[base + p];
                mk[p] = a.bslot[base + p];
            }
        }
        const uint64_t u = __ballot(s == ST_UNKNOWN), tk = __ballot(s == ST_TAKEN);
        if (lane == 0) {
            unk[w] = u;
            tak[w] = tk;
        }
    }
    __syncthreads();
    const uint64_t below = (1ull << lane) - 1ull;  // lanes before this one
    // members before the first changed position keep their state this sweep
    const int64_t ch0 = from <= (uint64_t)base ? 0 : (int64_t)((from - (uint64_t)base) >> 6);
    for (int64_t ch = ch0; ch < nw; ++ch) {
        uint64_t unk_ch = unk[ch];
        if (unk_ch == 0ull) continue;  // wave-uniform
        uint64_t tak_ch = tak[ch];
        const int64_t p = ch * kWave + lane;
        bool open = (unk_ch >> lane) & 1ull;  // still to decide in this sweep
        bool hit_tak_prev = false, hit_unk_prev = false;
        uint64_t own = 0ull;
        int64_t v = 0, l0 = 0;
        int k = 0;
        bool low_blocked = false;  // v's slots below k all known blocked when the chunk began
        if (open) {
            v = staged ? mv[p] : a.bmem[base + p];
            k = staged ? mk[p] : a.bslot[base + p];
            l0 = ir.loff + (v - ir.vstart) * T;
            // blocked bits only ever get set, so "all lower slots blocked" read
            // now stays true; if it reads false and the last lower slot is
            // blocked later, that blocker sets the ready byte and wakes this
            // bucket (slot k is then v's first open slot), and a later sweep
            // takes it
            low_blocked = k == 0 ||
                          __hip_atomic_load(&a.rdy[base + p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
            // earlier chunks are final for this sweep
            for (int64_t w = 0; w < ch; ++w) {
                const uint64_t r = Rm[p * nw + w];
                hit_tak_prev |= (r & tak[w]) != 0ull;
                hit_unk_prev |= (r & unk[w]) != 0ull;
            }
            own = Rm[p * nw + ch] & below;
        }
        // Settle the chunk in registers: no memory access between ballots.
        // act: 0 nothing, 1 slot blocked, 2 slot free and taken, 3 slot free
        // while v waits on lower slots (stays unknown here).
        int act = 0;
        while (true) {
            uint8_t ns = ST_UNKNOWN;
            if (open) {
                if (hit_tak_prev || (own & tak_ch)) {
                    ns = ST_NOT;
                    act = 1;
                } else if (!(hit_unk_prev || (own & unk_ch))) {
                    if (low_blocked) {
                        ns = ST_TAKEN;
                        act = 2;
                    } else {
                        act = 3;
                    }
                }
                if (act) open = false;
            }
            const uint64_t dec = __ballot(ns != ST_UNKNOWN);
            const uint64_t tk = __ballot(ns == ST_TAKEN);
            tak_ch |= tk;
            unk_ch &= ~dec;
            if (!dec) break;  // lanes still open wait on an undecided earlier member
        }
        // Publish the chunk's decisions: status bytes and colours, then the
        // per-vertex slot masks, failures and the wakes they imply (all lanes'
        // atomics in flight together).
        bool fin = false;  // v's colour (or failure) was decided here
        if (act) {
            const uint64_t kb = 1ull << (k & 63);
            if (act != 3)
                __hip_atomic_store(&a.st[base + p], act == 1 ? ST_NOT : ST_TAKEN, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            if (act == 2) {
                __hip_atomic_store(&a.col[v], (int32_t)c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                fin = true;
            }
            if (a.packed) {
                // blocked mask in bits 0-31, free mask in bits 32-63: one atomic
                // returns both (a blocked-slot count is their popcount)
                unsigned long long *w = (unsigned long long *)(a.blk + v);
                if (act == 1) {
                    const uint32_t bl = (uint32_t)atomicOr(w, (unsigned long long)kb) | (uint32_t)kb;
                    if (__popc(bl) == T) {  // the last slot was blocked
                        __hip_atomic_store(&a.col[v], COL_FAILED, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        fin = true;
                    } else {
                        const int f = __builtin_ctz(~bl);
                        if (f > k && f < T) ready_and_wake(a, l0 + f, out, out_count);
                    }
                } else {
                    const uint32_t fr = (uint32_t)(atomicOr(w, (unsigned long long)(kb << 32)) >> 32);
                    if (!(fr & (uint32_t)kb)) {
                        // as below: only k+1 .. (first free slot j) are new
                        int hi = T;
                        if (fr) {
                            const int j = __builtin_ctz(fr);
                            hi = j < k ? k : j + 1;
                        }
                        if (hi > k + 1) release_later_slots(a, l0, k, hi, out, out_count);
                    }
                }
            } else {
                uint64_t *blk = a.blk + v * a.fw;
                uint64_t *fre = a.fre + v * a.fw;
                if (act == 1) {
                    const uint64_t old = atomicOr((unsigned long long *)&blk[k >> 6], kb);
                    if (atomicAdd(&a.nblk[v], 1) == T - 1) {  // the last slot was blocked
                        __hip_atomic_store(&a.col[v], COL_FAILED, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        fin = true;
                    } else {
                        int f;
                        if (a.fw == 1) {
                            const uint64_t nb = ~(old | kb);
                            f = nb ? __builtin_ctzll(nb) : 64;
                        } else {
                            f = first_open(blk, T);
                        }
                        if (f > k && f < T) ready_and_wake(a, l0 + f, out, out_count);
                    }
                } else {
                    const uint64_t was = atomicOr((unsigned long long *)&fre[k >> 6], kb);
                    if (!(was & kb)) {
                        // the slots after the first slot j already found free
                        // were released then: only k+1 .. j are new (j itself
                        // stays unknown while v waits on lower slots, and v
                        // now takes k or an earlier slot); if j < k, nothing
                        int hi = T;
                        if (a.fw == 1 && was) {
                            const int j = __builtin_ctzll(was);
                            hi = j < k ? k : j + 1;
                        }
                        if (hi > k + 1) release_later_slots(a, l0, k, hi, out, out_count);
                    }
                }
            }
        }
        // decided vertices, counted once per chunk (one atomic per vertex on a
        // single counter serialises at this scale)
        const uint64_t fins = __ballot(fin);
        if (lane == 0 && fins)
            atomicAdd(&a.progress[(blockIdx.x % kJpSeg) * kJpProgStride], (unsigned long long)__popcll(fins));
        if (lane == 0) {
            tak[ch] = tak_ch;
            unk[ch] = unk_ch;
        }
        __syncthreads();
    }
}

// The sweep of a bucket of at most NW chunks whose vertices have lists of at
// most 32 colours (blocked and free masks in one word), with the rule of
// resolve_bucket and every memory access batched: the lane's member of each
// chunk (status, vertex, slot) in one set of loads; for the members still
// unknown, the list offset and length, the blocked mask and the relation row
// words of earlier chunks in a second; the chunks settle in registers; then
// all status bytes and colours are written, one slot-mask atomic per decided
// member is issued for every chunk before any result is used, and the
// failures, wakes and releases follow.
template <int NW>
__device__ void sweep_small(const JpArgs &a, int64_t c, int64_t base, int S, int nw, const uint64_t *Rm, uint64_t from,
                            int32_t *out, int32_t *out_count)
{
    const int lane = threadIdx.x;
    const uint64_t below = (1ull << lane) - 1ull;
    const int ch0 = from <= (uint64_t)base ? 0 : (int)((from - (uint64_t)base) >> 6);
    // the bucket's members share an instance: list size and list offsets from its record
    const InstRec &ir = a.inst[a.binst[c]];
    const int T = ir.T;
    uint8_t s[NW], rd[NW];
    uint32_t v[NW];
    int k[NW];
#pragma unroll
    for (int ch = 0; ch < NW; ++ch) {
        const int p = ch * kWave + lane;
        s[ch] = ST_NOT;
        rd[ch] = 0;
        v[ch] = 0u;
        k[ch] = 0;
        if (ch < nw && p < S) {
            s[ch] = __hip_atomic_load(&a.st[base + p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (ch >= ch0) {
                rd[ch] = __hip_atomic_load(&a.rdy[base + p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                v[ch] = a.bmem[base + p];
                k[ch] = a.bslot[base + p];
            }
        }
    }
    uint64_t unk[NW], tak[NW];
#pragma unroll
    for (int ch = 0; ch < NW; ++ch) {
        unk[ch] = __ballot(s[ch] == ST_UNKNOWN);
        tak[ch] = __ballot(s[ch] == ST_TAKEN);
    }
    uint64_t r[NW][NW];
#pragma unroll
    for (int ch = 0; ch < NW; ++ch) {
#pragma unroll
        for (int w = 0; w <= ch; ++w) r[ch][w] = 0ull;
        if (ch >= ch0 && ch < nw && s[ch] == ST_UNKNOWN) {
            const int64_t p = (int64_t)ch * kWave + lane;
#pragma unroll
            for (int w = 0; w <= ch; ++w) r[ch][w] = Rm[p * nw + w];
        }
    }
    // settle, chunk by chunk; act as in resolve_bucket
    int act[NW];
#pragma unroll
    for (int ch = 0; ch < NW; ++ch) {
        act[ch] = 0;
        if (ch < ch0 || ch >= nw || unk[ch] == 0ull) continue;  // wave-uniform
        uint64_t unk_ch = unk[ch], tak_ch = tak[ch];
        bool open = (unk_ch >> lane) & 1ull;
        bool hit_tak_prev = false, hit_unk_prev = false;
#pragma unroll
        for (int w = 0; w < ch; ++w) {
            hit_tak_prev |= (r[ch][w] & tak[w]) != 0ull;
            hit_unk_prev |= (r[ch][w] & unk[w]) != 0ull;
        }
        const uint64_t own = r[ch][ch] & below;
        // (ready bytes only ever get set: see resolve_bucket)
        const bool low_blocked = k[ch] == 0 || rd[ch] != 0;
        while (true) {
            uint8_t ns = ST_UNKNOWN;
            if (open) {
                if (hit_tak_prev || (own & tak_ch)) {
                    ns = ST_NOT;
                    act[ch] = 1;
                } else if (!(hit_unk_prev || (own & unk_ch))) {
                    if (low_blocked) {
                        ns = ST_TAKEN;
                        act[ch] = 2;
                    } else {
                        act[ch] = 3;
                    }
                }
                if (act[ch]) open = false;
            }
            const uint64_t dec = __ballot(ns != ST_UNKNOWN);
            tak_ch |= __ballot(ns == ST_TAKEN);
            unk_ch &= ~dec;
            if (!dec) break;
        }
        tak[ch] = tak_ch;
        unk[ch] = unk_ch;
    }
    // publish: status bytes and colours, then the slot-mask atomics
#pragma unroll
    for (int ch = 0; ch < NW; ++ch) {
        if (act[ch] == 1 || act[ch] == 2)
            __hip_atomic_store(&a.st[base + (int64_t)ch * kWave + lane], act[ch] == 1 ? ST_NOT : ST_TAKEN,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (act[ch] == 2) __hip_atomic_store(&a.col[v[ch]], (int32_t)c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    uint64_t old[NW];
#pragma unroll
    for (int ch = 0; ch < NW; ++ch) {
        old[ch] = 0ull;
        if (act[ch]) {
            const unsigned long long bit = 1ull << k[ch];
            old[ch] = atomicOr((unsigned long long *)(a.blk + v[ch]), act[ch] == 1 ? bit : bit << 32);
        }
    }
    int nfin = 0;
#pragma unroll
    for (int ch = 0; ch < NW; ++ch) {
        if (!act[ch]) continue;
        const uint32_t kb = 1u << k[ch];
        const int64_t l0 = ir.loff + ((int64_t)v[ch] - ir.vstart) * T;
        if (act[ch] == 2) ++nfin;
        if (act[ch] == 1) {
            const uint32_t bl = (uint32_t)old[ch] | kb;
            if (__popc(bl) == T) {  // the last slot was blocked
                __hip_atomic_store(&a.col[v[ch]], COL_FAILED, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ++nfin;
            } else {
                const int f = __builtin_ctz(~bl);
                if (f > k[ch] && f < T) ready_and_wake(a, l0 + f, out, out_count);
            }
        } else {
            const uint32_t fr = (uint32_t)(old[ch] >> 32);
            if (!(fr & kb)) {  // first free slot of v: release the later slots up to the next free one
                int hi = T;
                if (fr) {
                    const int j = __builtin_ctz(fr);
                    hi = j < k[ch] ? k[ch] : j + 1;
                }
                if (hi > k[ch] + 1) release_later_slots(a, l0, k[ch], hi, out, out_count);
            }
        }
    }
    // decided vertices of the sweep, one add per wave (nfin < 8)
    const unsigned long long n = __popcll(__ballot(nfin & 1)) + 2 * __popcll(__ballot(nfin & 2)) +
                                 4 * __popcll(__ballot(nfin & 4));
    if (lane == 0 && n) atomicAdd(&a.progress[(blockIdx.x % kJpSeg) * kJpProgStride], n);
}

constexpr int kJpSmallChunks = 4;  // buckets of at most 256 members take sweep_small

// One round of the worklist: visit the buckets listed by the previous round
// (wl[cur], segment lengths in counter row k); state changes append the
// buckets they may unblock to wl[cur ^ 1], counted in row k + 1.  No workgroup
// waits on another: rounds are separate launches in stream order.
__global__ void __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(6))) jp_round_kernel(JpArgs a, int cur,
                                                                                                   int32_t k)
{
    extern __shared__ uint64_t sbits[];  // taken[nw_max], unknown[nw_max]
    uint64_t *tak = sbits;
    uint64_t *unk = sbits + a.nw_max;
    __shared__ uint32_t mv[kJpStage];
    __shared__ slot_t mk[kJpStage];
    __shared__ unsigned long long from;
    __shared__ int32_t pre[kJpSeg + 1];  // segment starts of this round's list, and its length
    {
        // one wave: lane g holds segment g's length; inclusive prefix by shuffles
        const int g = threadIdx.x;
        int32_t x = g < kJpSeg ? a.wl_cnt[(int64_t)k * kJpRow + g * kJpCntStride] : 0;
        for (int d = 1; d < kWave; d <<= 1) {
            const int32_t y = __shfl_up(x, d, kWave);
            if (g >= d) x += y;
        }
        if (g < kJpSeg) pre[g + 1] = x;
        if (g == 0) pre[0] = 0;
        __syncthreads();
    }
    const int32_t n_in = pre[kJpSeg];
    int32_t *out = a.wl[cur ^ 1];
    int32_t *out_count = a.wl_cnt + (int64_t)(k + 1) * kJpRow;
    for (int64_t i = blockIdx.x; i < n_in; i += gridDim.x) {
        int lo = 0, hi = kJpSeg;  // pre[lo] <= i < pre[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (pre[mid] <= i) lo = mid;
            else hi = mid;
        }
        const int64_t c = a.wl[cur][lo * a.wl_cap + (i - pre[lo])];
        if (threadIdx.x == 0)
            from = __hip_atomic_exchange(&a.wake_at[c], kBusy, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        // a bucket woken again while it was swept is swept again at once
        for (int sweep = 0; sweep <= kJpResweeps && from < kBusy; ++sweep) {
            const int64_t base = a.bstart[c];
            const int64_t S = a.bstart[c + 1] - base;
            const int nwc = (int)((S + 63) >> 6);
            if (a.packed && nwc <= kJpSmallChunks)
                sweep_small<kJpSmallChunks>(a, c, base, (int)S, nwc, a.R + a.rb_off[c], from, out, out_count);
            else
                resolve_bucket(a, c, from, tak, unk, mv, mk, out, out_count);
            __syncthreads();
            if (threadIdx.x == 0)
                from = __hip_atomic_exchange(&a.wake_at[c], kBusy, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            if (from < kBusy) {
                // taken but not swept (resweep limit): the position goes back
                // and the bucket onto the next list
                atomicMin(&a.wake_at[c], from);
                append(a, c, out, out_count);
            } else if (atomicCAS(&a.wake_at[c], kBusy, kIdle) != kBusy) {
                // a position arrived after the last check (its waker found the
                // bucket busy and left the listing to this visit)
                append(a, c, out, out_count);
            }
        }
        __syncthreads();
    }
}

// Before a batch: slot 0 takes the current list length, the counters of the
// batch's rounds start at zero.  (A last-workgroup ticket that empties the
// consumed list inside each round was measured slower: 16384 workgroups per
// round on one counter cost about 80 us per round at n = 2M.)
__global__ void jp_batch_begin_kernel(int32_t *cnt, int32_t rounds)
{
    for (int32_t i = threadIdx.x; i < kJpSeg; i += blockDim.x)
        cnt[i * kJpCntStride] = cnt[(int64_t)kJpCountCell * kJpRow + i * kJpCntStride];
    for (int64_t i = threadIdx.x; i < (int64_t)rounds * kJpSeg; i += blockDim.x)
        cnt[(1 + i / kJpSeg) * kJpRow + (i % kJpSeg) * kJpCntStride] = 0;
}

// After a batch: its final lengths become the current ones; the totals the
// host reads (decided vertices, listed buckets) are summed here.  One wave.
__global__ void jp_batch_end_kernel(int32_t *cnt, int32_t rounds, const unsigned long long *progress,
                                    unsigned long long *totals)
{
    const int g = threadIdx.x;
    unsigned long long listed = 0, decided = 0;
    if (g < kJpSeg) {
        const int32_t n = cnt[(int64_t)rounds * kJpRow + g * kJpCntStride];
        cnt[(int64_t)kJpCountCell * kJpRow + g * kJpCntStride] = n;
        listed = (unsigned long long)n;
        decided = progress[g * kJpProgStride];
    }
    for (int d = kWave / 2; d > 0; d >>= 1) {
        listed += __shfl_down(listed, d, kWave);
        decided += __shfl_down(decided, d, kWave);
    }
    if (g == 0) {
        totals[0] = decided;
        totals[1] = listed;
    }
}

// Worklist of every bucket (the first round, and the host's recovery round).
__global__ void wl_all_kernel(int64_t P, int64_t cap, int32_t *wl, unsigned long long *wake_at, int32_t *cnt)
{
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < P; c += (int64_t)gridDim.x * blockDim.x) {
        wl[(c % kJpSeg) * cap + c / kJpSeg] = (int32_t)c;
        wake_at[c] = 0ull;  // listed, whole bucket
    }
    if (blockIdx.x == 0 && threadIdx.x < kJpSeg) {
        const int64_t g = threadIdx.x;
        cnt[(int64_t)kJpCountCell * kJpRow + g * kJpCntStride] = (int32_t)((P - g + kJpSeg - 1) / kJpSeg);
    }
}

// Relation bits of a bucket from a given symmetric CSR: for every edge
// {u, v} and every colour c in L(u) and L(v), set the pair's bits in bucket
// c (members located through pos_of[(vertex, slot)]).
__global__ void csr_to_relation_kernel(int64_t m, const int64_t *rowptr, const int32_t *adj, const uint32_t *lists,
                                       const int64_t *loff, const int64_t *pos_of, const int64_t *bstart,
                                       const int64_t *rb_off, uint64_t *R)
{
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < m; u += (int64_t)gridDim.x * blockDim.x) {
        const int64_t lu = loff[u];
        const int64_t Tu = loff[u + 1] - lu;
        const uint32_t *Lu = lists + lu;
        for (int64_t e = rowptr[u]; e < rowptr[u + 1]; ++e) {
            const int64_t v = adj[e];
            if (v == u) continue;
            const int64_t lv = loff[v];
            const int64_t Tv = loff[v + 1] - lv;
            const uint32_t *Lv = lists + lv;
            int64_t x = 0, y = 0;
            while (x < Tu && y < Tv) {
                if (Lu[x] == Lv[y]) {
                    const uint32_t c = Lu[x];
                    const int64_t S = bstart[c + 1] - bstart[c];
                    const int64_t nw = (S + 63) >> 6;
                    const int64_t pu = pos_of[lu + x] - bstart[c];
                    const int64_t pv = pos_of[lv + y] - bstart[c];
                    atomicOr((unsigned long long *)&R[rb_off[c] + pu * nw + (pv >> 6)], 1ull << (pv & 63));
                    ++x;
                    ++y;
                } else if (Lu[x] < Lv[y]) {
                    ++x;
                } else {
                    ++y;
                }
            }
        }
    }
}

__global__ void finish_kernel(Batch b, int64_t m, const int32_t *col, const int32_t *ids, int32_t *out_colors,
                              uint32_t *used_bits, unsigned long long *n_used, int32_t *uncol_flag)
{
    // The first vertex to set a colour's bit counts that colour for its
    // instance.  Those counts are summed over the wave before the atomic add
    // (one counter per instance would otherwise take one add per colour).
    const int lane = threadIdx.x & 63;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t c = col[i];
        int32_t ii = -1;
        bool first = false;
        if (c >= 0) {
            ii = b.vinst[i];
            const InstRec &r = b.inst[ii];
            if (out_colors) out_colors[ids[i]] = (int32_t)(r.cbase + (c - r.pal));
            const uint32_t bit = 1u << (c & 31);
            first = !(atomicOr(&used_bits[c >> 5], bit) & bit);
            uncol_flag[i] = 0;
        } else {
            uncol_flag[i] = 1;
        }
        const uint64_t firsts = __ballot(first);
        if (firsts) {
            const int lead = __builtin_ctzll(firsts);
            const int32_t lead_ii = __shfl(ii, lead, 64);
            const uint64_t same = __ballot(first && ii == lead_ii);
            if (lane == lead) atomicAdd(&n_used[lead_ii], (unsigned long long)__popcll(same));
            if (first && ii != lead_ii) atomicAdd(&n_used[ii], 1ull);
        }
    }
}

__global__ void compact_kernel(int64_t m, const int32_t *ids, const int32_t *flag, const int64_t *pos,
                               int32_t *next_ids)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        if (flag[i]) next_ids[pos[i]] = ids[i];
}

__global__ void instance_totals_kernel(Batch b, const int64_t *pos, const int64_t *rowptr, int64_t *m_next,
                                       int64_t *edges)
{
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < b.nb; i += gridDim.x * blockDim.x) {
        const InstRec &r = b.inst[i];
        if (m_next) m_next[i] = pos[r.vstart + r.m] - pos[r.vstart];
        if (edges) edges[i] = (rowptr[r.vstart + r.m] - rowptr[r.vstart]) / 2;
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

void launch_jp_all(const JpArgs &a, hipStream_t st)
{
    if (a.P <= 0) return;
    wl_all_kernel<<<grid_for(a.P, 256), 256, 0, st>>>(a.P, a.wl_cap, a.wl[0], a.wake_at, a.wl_cnt);
    PCHECK_LAUNCH();
}

void launch_jp_batch_begin(const JpArgs &a, int32_t rounds, hipStream_t st)
{
    if (rounds < 1 || rounds > kJpMaxBatch) throw Error(PICASSO_EINTERNAL, "colouring batch out of range");
    jp_batch_begin_kernel<<<1, 256, 0, st>>>(a.wl_cnt, rounds);
    PCHECK_LAUNCH();
}

void launch_jp_round(const JpArgs &a, int cur, int32_t k, hipStream_t st)
{
    if (a.P <= 0) return;
    if (k < 0 || k >= kJpMaxBatch) throw Error(PICASSO_EINTERNAL, "colouring round out of range");
    const size_t lds = (size_t)2 * a.nw_max * sizeof(uint64_t);
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(a.P, 16384));
    jp_round_kernel<<<(unsigned)grid, kWave, lds, st>>>(a, cur, k);
    PCHECK_LAUNCH();
}

void launch_jp_batch_end(const JpArgs &a, int32_t rounds, hipStream_t st)
{
    jp_batch_end_kernel<<<1, kWave, 0, st>>>(a.wl_cnt, rounds, a.progress, a.totals);
    PCHECK_LAUNCH();
}

void launch_csr_to_relation(int64_t m, const int64_t *rowptr, const int32_t *adj, const uint32_t *lists,
                            const int64_t *loff, const int64_t *pos_of, const int64_t *bstart, const int64_t *rb_off,
                            uint64_t *R, hipStream_t st)
{
    if (m <= 0) return;
    csr_to_relation_kernel<<<grid_for(m, 256), 256, 0, st>>>(m, rowptr, adj, lists, loff, pos_of, bstart, rb_off, R);
    PCHECK_LAUNCH();
}

void launch_finish_iteration(const Batch &b, int64_t m, const int32_t *col, const int32_t *ids, int32_t *out_colors,
                             uint32_t *used_bits, unsigned long long *n_used, int32_t *uncol_flag, hipStream_t st)
{
    if (m <= 0) return;
    finish_kernel<<<grid_for(m, 256), 256, 0, st>>>(b, m, col, ids, out_colors, used_bits, n_used, uncol_flag);
    PCHECK_LAUNCH();
}

void launch_instance_totals(const Batch &b, const int64_t *pos, const int64_t *rowptr, int64_t *m_next,
                            int64_t *edges, hipStream_t st)
{
    if (b.nb <= 0) return;
    instance_totals_kernel<<<grid_for(b.nb, 256), 256, 0, st>>>(b, pos, rowptr, m_next, edges);
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
