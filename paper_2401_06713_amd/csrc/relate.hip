// The relation between the members of a colour bucket (Sec. IV-A), as one
// S x S bit matrix R per bucket in HBM (row p holds ceil(S/64) words),
// symmetric: bit q of row p is set when members p and q fail the grouping
// relation.  Buckets are sorted by vertex priority, so member order is the
// colouring order.
//
// Popcount form (relate_kernel): with a = (x_u & z_v) ^ (z_u & x_v), bit k
// of a is set exactly when position k holds two different non-identity
// Paulis (Eq. 5).  ANTICOMMUTE: parity of popcount(a) (the parity rule of
// Sec. IV-A); QWC: a != 0.  int8 MFMA form: relate_mfma_kernel.
#include "common.h"

namespace picasso {
namespace {

constexpr int kWave = 64;

template <int W, int REL>
__device__ __forceinline__ uint32_t pair_bit(const uint32_t (&xi)[2 * W], const uint32_t (&zi)[2 * W],
                                             const uint32_t *xj, const uint32_t *zj)
{
    uint32_t acc = 0;
#pragma unroll
    for (int h = 0; h < 2 * W; ++h) {
        const uint32_t a = (xi[h] & zj[h]) ^ (zi[h] & xj[h]);
        if (REL == PICASSO_REL_QWC) acc |= a;
        else acc ^= a;
    }
    if (REL == PICASSO_REL_ANTICOMMUTE) return __popc(acc) & 1u;
    if (REL == PICASSO_REL_COMMUTE) return (__popc(acc) & 1u) ^ 1u;
    return acc != 0u;
}

// Members of a 64-wide tile t below the bucket size: the bits a row word may
// hold.  Padding members are zero strings, which commute with everything, so
// the COMMUTE relation masks them (the other relations give 0 there).
__device__ __forceinline__ uint64_t tile_mask(int64_t S, int64_t t)
{
    const int64_t k = S - t * 64;
    return k >= 64 ? ~0ull : ((1ull << k) - 1ull);
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

// LDS written by lanes of this wave becomes readable by its other lanes
// (a wave's LDS operations complete in order; this keeps the compiler from
// moving reads above the writes).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int W>
__device__ __forceinline__ void load_member(const uint64_t *bx, const uint64_t *bz, int64_t e, bool ok,
                                            uint32_t (&xo)[2 * W], uint32_t (&zo)[2 * W])
{
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const uint64_t xv = ok ? bx[e * W + w] : 0ull, zv = ok ? bz[e * W + w] : 0ull;
        xo[2 * w] = (uint32_t)xv;
        xo[2 * w + 1] = (uint32_t)(xv >> 32);
        zo[2 * w] = (uint32_t)zv;
        zo[2 * w + 1] = (uint32_t)(zv >> 32);
    }
}

// Each wave takes (bucket, row tile of 64 members) work items; 4 independent
// waves per workgroup.  Row members stay in registers; column members are
// staged in the wave's LDS slice.
//  - Diagonal tile: lane i tests column (i + s) mod 64 for s = 1..32, which
//    covers every pair of the tile at least once in 32 steps; the bits,
//    gathered at position s, are rotated into place and OR-ed with their
//    transpose.
//  - Tiles to the right: every lane reads the same column by broadcast;
//    lane i accumulates its row word, and a bit transpose gives the column
//    members' words, so each pair is tested once and written twice.
// Column blocks of 8 past the end of the bucket are skipped.
constexpr int kRelWaves = 4;

template <int W, int REL>
__global__ void __launch_bounds__(kWave * kRelWaves) relate_kernel(RelateArgs a)
{
    __shared__ uint32_t sx[kRelWaves][kWave * 2 * W], sz[kRelWaves][kWave * 2 * W];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t *cx = sx[wave], *cz = sz[wave];
    for (int64_t item = (int64_t)blockIdx.x * kRelWaves + wave; item < a.total_row_tiles;
         item += (int64_t)gridDim.x * kRelWaves) {
        const int64_t c = a.tile_bucket[item];
        const int64_t rt = item - a.tile_off[c];
        const int64_t base = a.bstart[c];
        const int64_t S = a.bstart[c + 1] - base;
        if (S <= a.mfma_max_members) continue;        // done by the MFMA kernel
        if (a.inst[a.binst[c]].rel != REL) continue;  // the other relation's launch
        const int64_t nw = (S + 63) >> 6;
        uint64_t *Rm = a.R + a.rb_off[c];
        const int64_t i = rt * kWave + lane;
        uint32_t xi[2 * W], zi[2 * W];
        load_member<W>(a.bx, a.bz, base + i, i < S, xi, zi);
        // diagonal tile
        wave_lds_sync();
#pragma unroll
        for (int h = 0; h < 2 * W; ++h) {
            cx[lane * 2 * W + h] = xi[h];
            cz[lane * 2 * W + h] = zi[h];
        }
        wave_lds_sync();
        uint32_t rl = 0u;
#pragma unroll 4
        for (int s = 1; s < 32; ++s) {
            const int jl = (lane + s) & 63;
            rl |= pair_bit<W, REL>(xi, zi, &cx[jl * 2 * W], &cz[jl * 2 * W]) << s;
        }
        const int j32 = (lane + 32) & 63;
        const uint64_t r = ((uint64_t)pair_bit<W, REL>(xi, zi, &cx[j32 * 2 * W], &cz[j32 * 2 * W]) << 32) | rl;
        const int rot = lane;
        const uint64_t placed = rot ? ((r << rot) | (r >> (64 - rot))) : r;
        uint64_t diag = placed | wave_transpose64(placed);
        if (REL == PICASSO_REL_COMMUTE) diag &= tile_mask(S, rt);
        if (i < S) Rm[i * nw + rt] = diag;
        // tiles to the right
        for (int64_t ct = rt + 1; ct < nw; ++ct) {
            const int64_t j = ct * kWave + lane;
            uint32_t xj[2 * W], zj[2 * W];
            load_member<W>(a.bx, a.bz, base + j, j < S, xj, zj);
            wave_lds_sync();
#pragma unroll
            for (int h = 0; h < 2 * W; ++h) {
                cx[lane * 2 * W + h] = xj[h];
                cz[lane * 2 * W + h] = zj[h];
            }
            wave_lds_sync();
            const int64_t cols = S - ct * kWave;
            const int blocks = cols >= kWave ? 8 : (int)((cols + 7) >> 3);
            uint64_t row = 0;
            for (int b = 0; b < blocks; ++b) {
                uint32_t bits8 = 0u;
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const int jj = b * 8 + t;
                    bits8 |= pair_bit<W, REL>(xi, zi, &cx[jj * 2 * W], &cz[jj * 2 * W]) << t;
                }
                row |= (uint64_t)bits8 << (b * 8);
            }
            if (REL == PICASSO_REL_COMMUTE) row &= tile_mask(S, ct);
            uint64_t col = wave_transpose64(row);
            if (REL == PICASSO_REL_COMMUTE) col &= tile_mask(S, rt);
            if (i < S) Rm[i * nw + ct] = row;
            if (j < S) Rm[j * nw + rt] = col;
        }
    }
}

// ---- int8 MFMA relation path ------------------------------------------------
// The relation as an integer matrix product.  Per qubit k, with 0/1 bytes:
//  ANTICOMMUTE: A_i = [x_i | z_i], B_j = [z_j | x_j];
//    (A B^T)[i][j] = sum_k x_ik z_jk + z_ik x_jk, whose parity is the
//    parity of the anticommuting positions (Eq. 5 and the parity rule).
//  QWC: A_i = [n_i | X_i | Y_i | Z_i] (n = non-identity, X/Y/Z one-hot),
//    B_j = [n_j | -X_j | -Y_j | -Z_j]; (A B^T)[i][j] = #(both non-identity)
//    - #(equal non-identity) > 0 exactly when some position holds two
//    different non-identity Paulis.
// One workgroup per bucket (buckets up to kMfmaMembers): the members are
// unpacked once into LDS rows of K bytes (each plane padded to a multiple of
// 16 qubits, so the swapped/negated B halves are contiguous 16-byte reads),
// then the four waves compute every 32 x 32 tile with
// v_mfma_i32_32x32x32_i8.  Lane l holds column j = l % 32 of a tile, i.e. by
// symmetry 16 bits of row j; two half-waves combine them into the row's
// 32-bit chunk for the tile's rows.  A and B fragments place bytes at the same
// (lane half, byte) positions, so the K order the hardware uses cancels out.
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
constexpr int kMfmaThreads = 256;
constexpr int kMfmaLds = 64 * 1024;   // bytes of unpacked member rows per bucket
constexpr int kMfmaMembers = 512;

// 4 bits of w starting at bit b -> 4 bytes of 0/1.
__device__ __forceinline__ uint32_t spread4(uint64_t w, int b)
{
    const uint32_t t = (uint32_t)(w >> b) & 0xFu;
    return (t * 0x00204081u) & 0x01010101u;
}

template <int REL>
__global__ void __launch_bounds__(kMfmaThreads) relate_mfma_kernel(RelateArgs a, int32_t qpad, int32_t kbytes)
{
    extern __shared__ uint32_t rows32[];  // S rows of kbytes
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int kd = kbytes >> 2;           // dwords per row
    for (int64_t c = blockIdx.x; c < a.P; c += gridDim.x) {
        const int64_t base = a.bstart[c];
        const int64_t S = a.bstart[c + 1] - base;
        if (S < 1 || S > a.mfma_max_members || a.inst[a.binst[c]].rel != REL) continue;
        if (S == 1) {  // a single member: its one row word holds no pair
            if (t == 0) a.R[a.rb_off[c]] = 0ull;
            continue;
        }
        const int nt = (int)((S + 31) >> 5);
        const int Sp = nt * 32;           // padded rows (zero strings)
        __syncthreads();
        // unpack: dword d of row r holds qubits 4d..4d+3 of one block
        for (int e = t; e < Sp * kd; e += kMfmaThreads) {
            const int r = e / kd, d = e - r * kd;
            uint32_t val = 0u;
            if (r < S) {
                const int blk = (4 * d) / qpad;          // which block of qpad bytes
                const int q0 = 4 * d - blk * qpad;       // first qubit of the dword
                const int w = q0 >> 6, b = q0 & 63;      // q0 % 4 == 0, so 4 bits stay in one word
                if (w < a.W) {
                    const uint64_t xv = a.bx[(base + r) * a.W + w], zv = a.bz[(base + r) * a.W + w];
                    if (REL != PICASSO_REL_QWC) {
                        val = spread4(blk == 0 ? xv : zv, b);
                    } else {
                        const uint64_t pick = blk == 0 ? (xv | zv) : blk == 1 ? (xv & ~zv) : blk == 2 ? (xv & zv) : (zv & ~xv);
                        val = spread4(pick, b);
                    }
                }
            }
            rows32[e] = val;
        }
        __syncthreads();
        const char *rows = reinterpret_cast<const char *>(rows32);
        const int half = lane >> 5, l32 = lane & 31;
        uint32_t *R32 = reinterpret_cast<uint32_t *>(a.R + a.rb_off[c]);
        const int64_t cpr = 2 * ((S + 63) >> 6);  // 32-bit chunks per row
        for (int tile = wave; tile < nt * nt; tile += kMfmaThreads / 64) {
            const int rt = tile / nt, ct = tile - rt * nt;
            const char *ra = rows + (int64_t)(rt * 32 + l32) * kbytes;
            const char *rb = rows + (int64_t)(ct * 32 + l32) * kbytes;
            v16i acc = {0};
            for (int kk = 0; kk < kbytes; kk += 32) {
                const int off = kk + 16 * half;
                const v4i av = *reinterpret_cast<const v4i *>(ra + off);
                v4i bv;
                if (REL != PICASSO_REL_QWC) {
                    const int boff = off < qpad ? off + qpad : off - qpad;  // [z | x]
                    bv = *reinterpret_cast<const v4i *>(rb + boff);
                } else {
                    bv = *reinterpret_cast<const v4i *>(rb + off);
                    if (off >= qpad) {
                        // 0/1 bytes -> 0/-1 bytes: spread bit 0 of each byte over
                        // its byte (no carry crosses a byte boundary)
                        bv |= bv << 1;
                        bv |= bv << 2;
                        bv |= bv << 4;
                    }
                }
                acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(av, bv, acc, 0, 0, 0);
            }
            // lane holds D[i][j] for column j = ct*32 + l32 and rows
            // i = rt*32 + 8*(r/4) + 4*half + r%4
            uint32_t m = 0u;
            const int64_t jcol = (int64_t)ct * 32 + l32;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int sh = 8 * (r >> 2) + 4 * half + (r & 3);
                uint32_t bitv;
                if (REL == PICASSO_REL_ANTICOMMUTE) bitv = (uint32_t)acc[r] & 1u;
                else if (REL == PICASSO_REL_QWC) bitv = acc[r] > 0 ? 1u : 0u;
                else {  // COMMUTE: even parity, except for a member with itself and padding rows
                    const int64_t irow = (int64_t)rt * 32 + sh;
                    bitv = (((uint32_t)acc[r] & 1u) ^ 1u) & (irow < S && irow != jcol ? 1u : 0u);
                }
                m |= bitv << sh;
            }
            m |= (uint32_t)__shfl_xor((int)m, 32, 64);
            const int64_t j = (int64_t)ct * 32 + l32;
            if (half == 0 && j < S) R32[j * cpr + rt] = m;
        }
        // the last chunk of a row past the padded tiles (odd tile count)
        if (nt & 1)
            for (int64_t j = t; j < S; j += kMfmaThreads) R32[j * cpr + nt] = 0u;
    }
}

// Strings of the bucket members in bucket order (one contiguous row per
// bucket entry), so the relation kernel's loads are coalesced.  Each member
// string is read from the interleaved copy (its W x words then its W z
// words, 16 W contiguous bytes): one random access per entry.
template <int W>
__global__ void gather_members_kernel(const uint32_t *__restrict__ bmem, int64_t entries,
                                      const int32_t *__restrict__ ids, const uint64_t *__restrict__ xz,
                                      uint64_t *__restrict__ bx, uint64_t *__restrict__ bz)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < entries;
         e += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t *src = xz + (int64_t)ids[bmem[e]] * (2 * W);
        uint64_t v[2 * W];
#pragma unroll
        for (int w = 0; w < 2 * W; ++w) v[w] = src[w];
#pragma unroll
        for (int w = 0; w < W; ++w) {
            bx[e * W + w] = v[w];
            bz[e * W + w] = v[W + w];
        }
    }
}

// x/z bit-planes -> per-string interleaved rows [x words | z words].
__global__ void interleave_kernel(const uint64_t *__restrict__ x, const uint64_t *__restrict__ z, int64_t n,
                                  int32_t W, uint64_t *__restrict__ xz)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        for (int w = 0; w < W; ++w) {
            xz[i * 2 * W + w] = x[i * W + w];
            xz[i * 2 * W + W + w] = z[i * W + w];
        }
}

// Owner bucket of every row tile.
__global__ void tile_bucket_kernel(const int64_t *__restrict__ tile_off, int64_t P, int32_t *__restrict__ owner)
{
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < P; c += (int64_t)gridDim.x * blockDim.x)
        for (int64_t t = tile_off[c]; t < tile_off[c + 1]; ++t) owner[t] = (int32_t)c;
}

unsigned grid_cap(int64_t items, int64_t cap = 1 << 22)
{
    if (items < 1) items = 1;
    return (unsigned)(items < cap ? items : cap);
}

}  // namespace

void launch_relate_prep(RelateArgs &a, int64_t entries, uint64_t *bx, uint64_t *bz, int32_t *tile_bucket,
                        hipStream_t st)
{
    if (entries > 0) {
        const unsigned grid = grid_cap((entries + 255) / 256, 65535 * 16);
        switch (a.W) {
            case 1: gather_members_kernel<1><<<grid, 256, 0, st>>>(a.bmem, entries, a.ids, a.xz, bx, bz); break;
            case 2: gather_members_kernel<2><<<grid, 256, 0, st>>>(a.bmem, entries, a.ids, a.xz, bx, bz); break;
            case 3: gather_members_kernel<3><<<grid, 256, 0, st>>>(a.bmem, entries, a.ids, a.xz, bx, bz); break;
            case 4: gather_members_kernel<4><<<grid, 256, 0, st>>>(a.bmem, entries, a.ids, a.xz, bx, bz); break;
            default: throw Error(PICASSO_EINTERNAL, "gather: unsupported word count");
        }
        PCHECK_LAUNCH();
    }
    if (a.P > 0) {
        tile_bucket_kernel<<<grid_cap((a.P + 255) / 256, 65535 * 16), 256, 0, st>>>(a.tile_off, a.P, tile_bucket);
        PCHECK_LAUNCH();
    }
    a.bx = bx;
    a.bz = bz;
    a.tile_bucket = tile_bucket;
}

void launch_relate(const RelateArgs &a, hipStream_t st)
{
    if (a.total_row_tiles <= 0) return;
    const unsigned grid = grid_cap((a.total_row_tiles + kRelWaves - 1) / kRelWaves);
#define PICASSO_REL_CASE(WW)                                                                       \
    case WW:                                                                                       \
        if (a.relation == PICASSO_REL_ANTICOMMUTE)                                                 \
            relate_kernel<WW, PICASSO_REL_ANTICOMMUTE><<<grid, kWave * kRelWaves, 0, st>>>(a);     \
        else if (a.relation == PICASSO_REL_COMMUTE)                                                \
            relate_kernel<WW, PICASSO_REL_COMMUTE><<<grid, kWave * kRelWaves, 0, st>>>(a);         \
        else                                                                                       \
            relate_kernel<WW, PICASSO_REL_QWC><<<grid, kWave * kRelWaves, 0, st>>>(a);             \
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

bool mfma_supported(int32_t q, int32_t relation)
{
    const int32_t qpad = (q + 15) / 16 * 16;
    const int32_t kbytes = relation == PICASSO_REL_QWC ? 4 * qpad : 2 * qpad;
    return kbytes % 32 == 0 && (int64_t)32 * kbytes <= kMfmaLds;
}

int64_t mfma_member_cap(int32_t q, int32_t relation)
{
    const int32_t qpad = (q + 15) / 16 * 16;
    const int32_t kbytes = relation == PICASSO_REL_QWC ? 4 * qpad : 2 * qpad;
    const int64_t fit = (int64_t)kMfmaLds / kbytes / 32 * 32;
    return fit < kMfmaMembers ? fit : kMfmaMembers;
}

void launch_relate_mfma(const RelateArgs &a, int32_t q, hipStream_t st)
{
    if (a.P <= 0) return;
    const int32_t qpad = (q + 15) / 16 * 16;
    const int32_t kbytes = a.relation == PICASSO_REL_QWC ? 4 * qpad : 2 * qpad;
    // member rows of the largest bucket this launch takes (at most the LDS cap)
    const int64_t cap = std::min<int64_t>(mfma_member_cap(q, a.relation), std::max<int64_t>(a.mfma_max_members, 1));
    const size_t lds = (size_t)((cap + 31) / 32 * 32) * kbytes;
    const unsigned grid = grid_cap(a.P, 1 << 20);
    if (a.relation == PICASSO_REL_ANTICOMMUTE)
        relate_mfma_kernel<PICASSO_REL_ANTICOMMUTE><<<grid, kMfmaThreads, lds, st>>>(a, qpad, kbytes);
    else if (a.relation == PICASSO_REL_COMMUTE)
        relate_mfma_kernel<PICASSO_REL_COMMUTE><<<grid, kMfmaThreads, lds, st>>>(a, qpad, kbytes);
    else
        relate_mfma_kernel<PICASSO_REL_QWC><<<grid, kMfmaThreads, lds, st>>>(a, qpad, kbytes);
    PCHECK_LAUNCH();
}

void launch_interleave(const uint64_t *x, const uint64_t *z, int64_t n, int32_t W, uint64_t *xz, hipStream_t st)
{
    if (n <= 0) return;
    interleave_kernel<<<grid_cap((n + 255) / 256, 65535 * 16), 256, 0, st>>>(x, z, n, W, xz);
    PCHECK_LAUNCH();
}

}  // namespace picasso
