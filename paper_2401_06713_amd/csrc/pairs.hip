// Intra-bucket pair kernels: the conflict-graph build (Alg. 1
// construct_conflict_graph; Sec. IV-A; the output CSR of Alg. 3).
//
// A pair {u, v} conflicts iff the relation holds and L(u), L(v) share a
// colour.  Every such pair lies in the bucket of each shared colour, so the
// kernels visit the pairs of each bucket and keep a pair only in the bucket
// of its smallest shared colour c: L(u) and L(v) are sorted, so "no smaller
// shared colour" means the list prefixes before c are disjoint.
//
// Relation, popcount form: with a = (x_u & z_v) ^ (z_u & x_v), bit k of a is
// 1 exactly when position k holds two different non-identity Paulis
// (Eq. 5).  ANTICOMMUTE: parity of popcount(a) (the parity rule of
// Sec. IV-A).  QWC: a != 0.
//
// Count pass: exact per-vertex degrees.  Fill pass: the same enumeration
// writes each edge into both endpoints' CSR rows at positions claimed from
// per-vertex cursors.
#include "common.h"

namespace picasso {
namespace {

constexpr int kThreads = 256;
constexpr int kChunk = 512;  // bucket members staged in LDS per column chunk

template <int W, int REL>
__device__ __forceinline__ bool relation_holds(const uint64_t *xi, const uint64_t *zi, const uint64_t *xj,
                                               const uint64_t *zj)
{
    uint64_t acc = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const uint64_t a = (xi[w] & zj[w]) ^ (zi[w] & xj[w]);
        if (REL == PICASSO_REL_ANTICOMMUTE) acc ^= a;
        else acc |= a;
    }
    if (REL == PICASSO_REL_ANTICOMMUTE) return (__popcll(acc) & 1) != 0;
    return acc != 0;
}

// True when the sorted prefixes La[0..ka) and Lb[0..kb) share a colour,
// i.e. the pair shares a colour smaller than the current bucket's.
__device__ __forceinline__ bool prefixes_intersect(const uint32_t *La, int ka, const uint32_t *Lb, int kb)
{
    int a = 0, b = 0;
    while (a < ka && b < kb) {
        const uint32_t ca = La[a], cb = Lb[b];
        if (ca == cb) return true;
        a += ca < cb;
        b += cb < ca;
    }
    return false;
}

template <int W, int REL, bool FILL>
__global__ void __launch_bounds__(kThreads) pair_kernel(PairArgs a)
{
    __shared__ uint64_t sx[kChunk * W], sz[kChunk * W];
    __shared__ uint32_t su[kChunk];
    __shared__ uint8_t sk[kChunk];
    const int t = threadIdx.x;
    for (int64_t c = blockIdx.x; c < a.P; c += gridDim.x) {
        const int64_t base = a.bstart[c];
        const int64_t S = a.bstart[c + 1] - base;
        if (S < 2) continue;
        for (int64_t r0 = 0; r0 < S; r0 += kThreads) {
            const int64_t i = r0 + t;
            uint64_t xi[W], zi[W];
            uint32_t ui = 0;
            int ki = 0;
            if (i < S) {
                ui = a.bmem[base + i];
                ki = a.bslot[base + i];
                const int64_t g = (int64_t)a.ids[ui] * W;
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    xi[w] = a.x[g + w];
                    zi[w] = a.z[g + w];
                }
            }
            for (int64_t c0 = r0; c0 < S; c0 += kChunk) {
                const int64_t cn = (S - c0) < kChunk ? (S - c0) : kChunk;
                __syncthreads();
                for (int64_t e = t; e < cn; e += kThreads) {
                    const uint32_t u = a.bmem[base + c0 + e];
                    su[e] = u;
                    sk[e] = a.bslot[base + c0 + e];
                    const int64_t g = (int64_t)a.ids[u] * W;
#pragma unroll
                    for (int w = 0; w < W; ++w) {
                        sx[e * W + w] = a.x[g + w];
                        sz[e * W + w] = a.z[g + w];
                    }
                }
                __syncthreads();
                if (i < S) {
                    int64_t jb = i + 1 - c0;
                    if (jb < 0) jb = 0;
                    for (int64_t jj = jb; jj < cn; ++jj) {
                        if (!relation_holds<W, REL>(xi, zi, &sx[jj * W], &sz[jj * W])) continue;
                        const uint32_t uj = su[jj];
                        const int kj = sk[jj];
                        if (ki > 0 && kj > 0 &&
                            prefixes_intersect(a.lists + (int64_t)ui * a.T, ki, a.lists + (int64_t)uj * a.T, kj))
                            continue;
                        if (!FILL) {
                            atomicAdd(&a.deg[ui], 1);
                            atomicAdd(&a.deg[uj], 1);
                        } else {
                            const int pi = atomicAdd(&a.cursor[ui], 1);
                            const int pj = atomicAdd(&a.cursor[uj], 1);
                            a.adj[a.rowptr[ui] + pi] = (int32_t)uj;
                            a.adj[a.rowptr[uj] + pj] = (int32_t)ui;
                        }
                    }
                }
            }
        }
    }
}

template <bool FILL>
void launch(const PairArgs &a, hipStream_t st)
{
    if (a.P <= 0) return;
    const unsigned grid = (unsigned)(a.P < (1 << 20) ? a.P : (1 << 20));
#define PICASSO_PAIR_CASE(WW)                                                                      \
    case WW:                                                                                       \
        if (a.relation == PICASSO_REL_ANTICOMMUTE)                                                 \
            pair_kernel<WW, PICASSO_REL_ANTICOMMUTE, FILL><<<grid, kThreads, 0, st>>>(a);          \
        else                                                                                       \
            pair_kernel<WW, PICASSO_REL_QWC, FILL><<<grid, kThreads, 0, st>>>(a);                  \
        break;
    switch (a.W) {
        PICASSO_PAIR_CASE(1)
        PICASSO_PAIR_CASE(2)
        PICASSO_PAIR_CASE(3)
        PICASSO_PAIR_CASE(4)
        default:
            throw Error(PICASSO_EINTERNAL, "pair kernel: unsupported word count");
    }
#undef PICASSO_PAIR_CASE
    PCHECK_LAUNCH();
}

}  // namespace

void launch_pair_count(const PairArgs &a, hipStream_t st) { launch<false>(a, st); }
void launch_pair_fill(const PairArgs &a, hipStream_t st) { launch<true>(a, st); }

}  // namespace picasso
