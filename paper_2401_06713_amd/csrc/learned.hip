// Learned parameters: instance features and the predictor network.
//
// The paper chooses (palette %, alpha) with a regressor trained on parameter
// sweeps and given the graph and the trade-off weight beta of its
// bi-objective (Sec. VI, Eq. 7).  Here a 3-layer perceptron 6 -> 64 -> 64 -> 2
// (ReLU hidden layers, FP32) maps five features of the current iteration
// (ln m, q, mean Pauli weight, sampled relation density, iteration) and beta
// to (f, alpha) = (0.01 + 0.24 sigmoid(o0), 1 + 3 sigmoid(o1)).
//
// Parameter vector layout (4738 floats): W1[64][6], b1[64], W2[64][64],
// b2[64], W3[2][64], b3[2].  Inputs are scaled by (1/16, 1/128, 1/128, 1,
// 1/16, 1) before the first layer.  Training loss over B rows:
// (1/(2B)) sum (o - t)^2, minimised with Adam.
#include <algorithm>

#include "common.h"

namespace picasso {
namespace {

constexpr int H = kMlpHidden, NI = kMlpIn, NO = kMlpOut;
constexpr int OFF_B1 = H * NI, OFF_W2 = OFF_B1 + H, OFF_B2 = OFF_W2 + H * H, OFF_W3 = OFF_B2 + H,
              OFF_B3 = OFF_W3 + NO * H;
constexpr uint32_t TAG_FEAT = 0x46454154u;

// ---- features -------------------------------------------------------------
// Sum of Pauli weights (non-identity positions) over the current vertices,
// and the number of K sampled ordered pairs of distinct vertices joined by
// the relation.  Pair k: a = floor(r1 m / 2^64), b' = floor(r2 (m-1) / 2^64),
// b = b' + (b' >= a), r1, r2 = the keyed draws (seed; k, 0|1, ell, "FEAT").
__global__ void features_kernel(int64_t m, const int32_t *__restrict__ ids, const uint64_t *__restrict__ x,
                                const uint64_t *__restrict__ z, int32_t W, uint64_t seed, uint32_t ell, int32_t rel,
                                int32_t K, unsigned long long *__restrict__ weight, unsigned long long *__restrict__ hits)
{
    unsigned long long wsum = 0, hsum = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
        const int64_t g = (int64_t)ids[i] * W;
        for (int w = 0; w < W; ++w) wsum += __popcll(x[g + w] | z[g + w]);
    }
    if (m >= 2)
        for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < K; k += stride) {
            const uint64_t r1 = philox_draw(seed, (uint32_t)k, 0, ell, TAG_FEAT);
            const uint64_t r2 = philox_draw(seed, (uint32_t)k, 1, ell, TAG_FEAT);
            const uint64_t a = __umul64hi(r1, (uint64_t)m);
            uint64_t b = __umul64hi(r2, (uint64_t)(m - 1));
            if (b >= a) ++b;
            const int64_t ga = (int64_t)ids[a] * W, gb = (int64_t)ids[b] * W;
            uint64_t par = 0, any = 0;
            for (int w = 0; w < W; ++w) {
                const uint64_t t = (x[ga + w] & z[gb + w]) ^ (z[ga + w] & x[gb + w]);
                par ^= t;
                any |= t;
            }
            const unsigned long long odd = __popcll(par) & 1;
            hsum += rel == PICASSO_REL_ANTICOMMUTE ? odd : rel == PICASSO_REL_COMMUTE ? 1 - odd : (any != 0);
        }
    for (int d = 32; d > 0; d >>= 1) {
        wsum += __shfl_down(wsum, d, 64);
        hsum += __shfl_down(hsum, d, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        if (wsum) atomicAdd(weight, wsum);
        if (hsum) atomicAdd(hits, hsum);
    }
}

// Relation density of each instance of a batch (the conflict-graph size
// prediction): block (kb, a) tests pairs kb*256 .. kb*256+255 of instance a,
// drawn as in features_kernel from the instance's seed.
__global__ void density_kernel(Batch b, const int32_t *__restrict__ ids, const uint64_t *__restrict__ x,
                               const uint64_t *__restrict__ z, int32_t W, uint32_t ell, int32_t K,
                               uint32_t *__restrict__ hits)
{
    for (int32_t ai = blockIdx.y; ai < b.nb; ai += gridDim.y) {
        const InstRec &r = b.inst[ai];
        const int64_t m = r.m;
        const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        uint32_t hit = 0;
        if (m >= 2 && k < K) {
            const uint64_t r1 = philox_draw(r.seed, (uint32_t)k, 0, ell, TAG_FEAT);
            const uint64_t r2 = philox_draw(r.seed, (uint32_t)k, 1, ell, TAG_FEAT);
            const uint64_t pa = __umul64hi(r1, (uint64_t)m);
            uint64_t pb = __umul64hi(r2, (uint64_t)(m - 1));
            if (pb >= pa) ++pb;
            const int64_t ga = (int64_t)ids[r.vstart + pa] * W, gb = (int64_t)ids[r.vstart + pb] * W;
            uint64_t par = 0, any = 0;
            for (int w = 0; w < W; ++w) {
                const uint64_t t = (x[ga + w] & z[gb + w]) ^ (z[ga + w] & x[gb + w]);
                par ^= t;
                any |= t;
            }
            const uint32_t odd = __popcll(par) & 1;
            hit = r.rel == PICASSO_REL_ANTICOMMUTE ? odd : r.rel == PICASSO_REL_COMMUTE ? 1 - odd : (any != 0);
        }
        const uint64_t bal = __ballot(hit != 0);
        if ((threadIdx.x & 63) == 0 && bal) atomicAdd(&hits[ai], (uint32_t)__popcll(bal));
    }
}

// ---- the network ----------------------------------------------------------
__device__ __forceinline__ void scale_inputs(const float *raw, float *xin)
{
    xin[0] = raw[0] * (1.0f / 16.0f);
    xin[1] = raw[1] * (1.0f / 128.0f);
    xin[2] = raw[2] * (1.0f / 128.0f);
    xin[3] = raw[3];
    xin[4] = raw[4] * (1.0f / 16.0f);
    xin[5] = raw[5];
}

// One thread per row.  Keeps what the gradient needs when `keep` is set:
// per row xin[5], h1[64], h2[64], d3[2], d2[64], d1[64] (the back-propagated
// deltas of the loss against targets t).
__global__ void __launch_bounds__(128) mlp_rows_kernel(const float *__restrict__ p, const float *__restrict__ raw,
                                                       int32_t B, float *__restrict__ out,
                                                       const float *__restrict__ target, float *__restrict__ keep,
                                                       float *__restrict__ row_loss)
{
    __shared__ float sp[kMlpParams];
    for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) sp[i] = p[i];
    __syncthreads();
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    float xin[NI], h1[H], h2[H], o[NO];
    scale_inputs(raw + (int64_t)b * NI, xin);
    for (int j = 0; j < H; ++j) {
        float s = sp[OFF_B1 + j];
        for (int i = 0; i < NI; ++i) s = fmaf(sp[j * NI + i], xin[i], s);
        h1[j] = s > 0.f ? s : 0.f;
    }
    for (int j = 0; j < H; ++j) {
        float s = sp[OFF_B2 + j];
        for (int i = 0; i < H; ++i) s = fmaf(sp[OFF_W2 + j * H + i], h1[i], s);
        h2[j] = s > 0.f ? s : 0.f;
    }
    for (int k = 0; k < NO; ++k) {
        float s = sp[OFF_B3 + k];
        for (int i = 0; i < H; ++i) s = fmaf(sp[OFF_W3 + k * H + i], h2[i], s);
        o[k] = s;
    }
    if (out)
        for (int k = 0; k < NO; ++k) out[(int64_t)b * NO + k] = o[k];
    if (!keep) return;
    float *kp = keep + (int64_t)b * kMlpKeep;
    float d3[NO];
    float loss = 0.f;
    for (int k = 0; k < NO; ++k) {
        const float e = o[k] - target[(int64_t)b * NO + k];
        loss += 0.5f * e * e;
        d3[k] = e / (float)B;
    }
    row_loss[b] = loss / (float)B;
    float d2[H];
    for (int i = 0; i < H; ++i) {
        float s = 0.f;
        for (int k = 0; k < NO; ++k) s = fmaf(sp[OFF_W3 + k * H + i], d3[k], s);
        d2[i] = h2[i] > 0.f ? s : 0.f;
    }
    for (int i = 0; i < NI; ++i) kp[i] = xin[i];
    for (int i = 0; i < H; ++i) {
        float s = 0.f;
        for (int j = 0; j < H; ++j) s = fmaf(sp[OFF_W2 + j * H + i], d2[j], s);
        kp[NI + i] = h1[i];
        kp[NI + H + i] = h2[i];
        kp[NI + 2 * H + NO + H + i] = h1[i] > 0.f ? s : 0.f;  // d1
        kp[NI + 2 * H + NO + i] = d2[i];
    }
    for (int k = 0; k < NO; ++k) kp[NI + 2 * H + k] = d3[k];
}

// Gradient of every parameter: one thread per parameter, summing its
// per-row contributions in row order (deterministic).
__global__ void mlp_grad_kernel(const float *__restrict__ keep, int32_t B, float *__restrict__ grad)
{
    const int pidx = blockIdx.x * blockDim.x + threadIdx.x;
    if (pidx >= kMlpParams) return;
    const int XIN = 0, H1 = NI, H2 = NI + H, D3 = NI + 2 * H, D2 = D3 + NO, D1 = D2 + H;
    int dsel, dj, asel, ai;  // grad = sum_rows delta[dsel + dj] * act[asel + ai] (act = 1 for biases)
    if (pidx < OFF_B1) {
        dsel = D1, dj = pidx / NI, asel = XIN, ai = pidx % NI;
    } else if (pidx < OFF_W2) {
        dsel = D1, dj = pidx - OFF_B1, asel = -1, ai = 0;
    } else if (pidx < OFF_B2) {
        dsel = D2, dj = (pidx - OFF_W2) / H, asel = H1, ai = (pidx - OFF_W2) % H;
    } else if (pidx < OFF_W3) {
        dsel = D2, dj = pidx - OFF_B2, asel = -1, ai = 0;
    } else if (pidx < OFF_B3) {
        dsel = D3, dj = (pidx - OFF_W3) / H, asel = H2, ai = (pidx - OFF_W3) % H;
    } else {
        dsel = D3, dj = pidx - OFF_B3, asel = -1, ai = 0;
    }
    float s = 0.f;
    for (int b = 0; b < B; ++b) {
        const float *kp = keep + (int64_t)b * kMlpKeep;
        s = fmaf(kp[dsel + dj], asel < 0 ? 1.f : kp[asel + ai], s);
    }
    grad[pidx] = s;
}

__global__ void adam_kernel(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m1,
                            float *__restrict__ m2, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kMlpParams) return;
    const float gi = g[i];
    const float mi = b1 * m1[i] + (1.f - b1) * gi;
    const float vi = b2 * m2[i] + (1.f - b2) * gi * gi;
    m1[i] = mi;
    m2[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void squash_kernel(const float *__restrict__ o, int32_t B, float *__restrict__ fa)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    fa[2 * b] = 0.01f + 0.24f / (1.f + expf(-o[2 * b]));
    fa[2 * b + 1] = 1.f + 3.f / (1.f + expf(-o[2 * b + 1]));
}

}  // namespace

void launch_features(int64_t m, const int32_t *ids, const uint64_t *x, const uint64_t *z, int32_t W, uint64_t seed,
                     uint32_t ell, int32_t rel, int32_t K, unsigned long long *weight, unsigned long long *hits,
                     hipStream_t st)
{
    int64_t work = m > K ? m : K;
    int64_t blocks = (work + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 4096) blocks = 4096;
    features_kernel<<<(unsigned)blocks, 256, 0, st>>>(m, ids, x, z, W, seed, ell, rel, K, weight, hits);
    PCHECK_LAUNCH();
}

void launch_density(const Batch &b, const int32_t *ids, const uint64_t *x, const uint64_t *z, int32_t W, uint32_t ell,
                    int32_t K, uint32_t *hits, hipStream_t st)
{
    if (b.nb <= 0 || K <= 0) return;
    const dim3 grid((unsigned)((K + 255) / 256), (unsigned)std::min<int32_t>(b.nb, 65535));
    density_kernel<<<grid, 256, 0, st>>>(b, ids, x, z, W, ell, K, hits);
    PCHECK_LAUNCH();
}

void launch_mlp_rows(const float *p, const float *raw, int32_t B, float *out, const float *target, float *keep,
                     float *row_loss, hipStream_t st)
{
    if (B <= 0) return;
    mlp_rows_kernel<<<(unsigned)((B + 127) / 128), 128, 0, st>>>(p, raw, B, out, target, keep, row_loss);
    PCHECK_LAUNCH();
}

void launch_mlp_grad(const float *keep, int32_t B, float *grad, hipStream_t st)
{
    mlp_grad_kernel<<<(kMlpParams + 255) / 256, 256, 0, st>>>(keep, B, grad);
    PCHECK_LAUNCH();
}

void launch_adam(float *p, const float *g, float *m1, float *m2, float lr, float b1, float b2, float eps, int32_t step,
                 hipStream_t st)
{
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    adam_kernel<<<(kMlpParams + 255) / 256, 256, 0, st>>>(p, g, m1, m2, lr, b1, b2, eps, c1, c2);
    PCHECK_LAUNCH();
}

void launch_squash(const float *o, int32_t B, float *fa, hipStream_t st)
{
    if (B <= 0) return;
    squash_kernel<<<(unsigned)((B + 255) / 256), 256, 0, st>>>(o, B, fa);
    PCHECK_LAUNCH();
}

}  // namespace picasso
