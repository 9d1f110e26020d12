// cae_mlp.hip -- bfloat16 matrix-core training and inference kernels of the calibration surrogate.
//
// The surrogate is a multilayer perceptron d_in -> H -> H -> d_out with SiLU hidden activations
// that maps agent-population parameters to ensemble statistics.  It is not part of the paper's
// method; it accelerates the parameter sweeps the paper motivates (section IV-J) and the exact
// engine stays its fallback and the reference that measures its error.
//
// Precision: weights, inputs, hidden activations and back-propagated gradients are stored in
// bfloat16 (round to nearest even); every product is accumulated in fp32 on the matrix cores
// (v_mfma_f32_16x16x16bf16_1k in the general GEMM and the fused inference kernel, gfx950's
// v_mfma_f32_16x16x32_bf16 in the fused training step); biases, pre-activations, outputs, weight
// gradients and the Adam state are fp32.  Parameter layout (row-major, input index first):
//   W1[d_in][H], b1[H], W2[H][H], b2[H], W3[H][d_out], b3[d_out]
// and the bfloat16 weight copies are W1, W2, W3 in the same layouts, back to back, followed by
// W2 transposed (W2T[n][k] = W2[k][n]) for the fused inference kernel, whose matrix-core
// operands want four consecutive input indices per lane.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <mutex>

#include "cae.h"

namespace {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f)  // round to nearest even
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)(u >> 16);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float silu(float z) { return z / (1.0f + expf(-z)); }

__device__ __forceinline__ float dsilu(float z)
{
    const float s = 1.0f / (1.0f + expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

enum Epi : int {
    EPI_HIDDEN = 0,  // z = acc + bias -> Z (f32), H = bf16(silu(z))
    EPI_OUTPUT = 1,  // y = acc + bias -> f32
    EPI_DSILU = 2,   // dz = bf16(acc * silu'(Z))
    EPI_F32 = 3,     // acc -> f32
};

struct GemmArgs {
    const uint16_t *A;  // bf16, M x K (or K x M when transposed)
    const uint16_t *B;  // bf16, K x N (or N x K when transposed)
    uint32_t lda, ldb;
    uint32_t M, N, K;
    uint32_t ones_row;  // A has one extra row M of ones (its output row is the column sum of B)
    uint32_t kchunk;    // K range per blockIdx.y (split K); partial sums go to Of + y * (M+1) * ldo
    const float *bias;  // EPI_HIDDEN / EPI_OUTPUT
    const float *Zin;   // EPI_DSILU: pre-activations (M x N, ld = ldo)
    float *Of;          // f32 output (Z, y, or gradient), ld = ldo
    uint16_t *Ob;       // bf16 output (H or dz), ld = ldo
    uint32_t ldo;
};

// C = A * B with one wave per 16x16 output tile (four tiles per workgroup).  MFMA operand
// layout (16x16x16): lane l holds A[l%16][4*(l/16)+t] and B[4*(l/16)+t][l%16], t = 0..3, and
// receives C[4*(l/16)+t][l%16].
template <bool TA, bool TB, int EPI>
__global__ void __launch_bounds__(256) mlp_gemm(const GemmArgs g)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = threadIdx.x >> 6;
    const uint32_t Mr = g.M + g.ones_row;  // rows of the output
    const uint32_t tiles_n = (g.N + 15u) / 16u;
    const uint32_t tile = blockIdx.x * 4u + wave;
    const uint32_t ti = tile / tiles_n, tj = tile % tiles_n;
    if (ti * 16u >= Mr) return;
    const uint32_t r = lane & 15u, grp = lane >> 4;
    const uint32_t row = ti * 16u + r;  // A row this lane feeds
    const uint32_t col = tj * 16u + r;  // B column this lane feeds
    const uint32_t kbeg = blockIdx.y * g.kchunk;
    const uint32_t kend = min(g.K, kbeg + g.kchunk);
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    for (uint32_t k0 = kbeg; k0 < kend; k0 += 16u) {
        v4s a, b;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const uint32_t k = k0 + 4u * grp + (uint32_t)t;
            uint16_t av = 0, bv = 0;
            if (k < kend) {
                if (row < g.M) av = TA ? g.A[(size_t)k * g.lda + row] : g.A[(size_t)row * g.lda + k];
                else if (row == g.M && g.ones_row) av = 0x3F80u;  // bfloat16 1.0
                if (col < g.N) bv = TB ? g.B[(size_t)col * g.ldb + k] : g.B[(size_t)k * g.ldb + col];
            }
            a[t] = (short)av;
            b[t] = (short)bv;
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
    const uint32_t j = tj * 16u + r;
    if (j >= g.N) return;
    float *Of = g.Of + (size_t)blockIdx.y * Mr * g.ldo;  // split-K partial (y = 0 when not split)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const uint32_t i = ti * 16u + 4u * grp + (uint32_t)t;
        if (i >= Mr) continue;
        const size_t o = (size_t)i * g.ldo + j;
        if constexpr (EPI == EPI_HIDDEN) {
            const float z = acc[t] + g.bias[j];
            g.Of[o] = z;
            g.Ob[o] = f2bf(silu(z));
        } else if constexpr (EPI == EPI_OUTPUT) {
            g.Of[o] = acc[t] + g.bias[j];
        } else if constexpr (EPI == EPI_DSILU) {
            g.Ob[o] = f2bf(acc[t] * dsilu(g.Zin[o]));
        } else {
            Of[o] = acc[t];
        }
    }
}

// out[i] = sum over the `parts` split-K partial results, in partial order (deterministic).
__global__ void sum_partials(const float *part, uint32_t parts, uint64_t n, float *out)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        float s = 0.f;
        for (uint32_t p = 0; p < parts; ++p) s += part[(size_t)p * n + i];
        out[i] = s;
    }
}

__global__ void to_bf16(const float *x, uint16_t *y, uint64_t n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        y[i] = f2bf(x[i]);
}

// Mean loss over n values and its gradient, one workgroup, fixed reduction order.
//   kind 0 (squared error): loss = mean r^2,                         dy = 2 r / n
//   kind 1 (Huber, delta):  loss = mean(r^2/2 if |r| <= delta else delta (|r| - delta/2)),
//                           dy = clamp(r, -delta, delta) / n
// with r = y - t.
__global__ void __launch_bounds__(1024) loss_grad(const float *y, const float *t, float *dy, float *loss, uint32_t n,
                                                  int kind, float delta)
{
    __shared__ float part[1024];
    float s = 0.f;
    const float inv = 1.0f / (float)n;
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
        const float d = y[i] - t[i];
        if (kind == 0) {
            dy[i] = 2.0f * d * inv;
            s += d * d;
        } else {
            const float a = fabsf(d);
            dy[i] = fminf(fmaxf(d, -delta), delta) * inv;
            s += a <= delta ? 0.5f * d * d : delta * (a - 0.5f * delta);
        }
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (uint32_t w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = part[0] / (float)n;
}

struct Layout {
    uint64_t w1, b1, w2, b2, w3, b3, P;  // param offsets
    uint64_t w2t;                        // bf16 offset of the transposed W2 copy
    uint64_t W;                          // bf16 weight count
};

__host__ __device__ inline Layout layout(uint32_t din, uint32_t H, uint32_t dout)
{
    Layout l;
    l.w1 = 0;
    l.b1 = l.w1 + (uint64_t)din * H;
    l.w2 = l.b1 + H;
    l.b2 = l.w2 + (uint64_t)H * H;
    l.w3 = l.b2 + H;
    l.b3 = l.w3 + (uint64_t)H * dout;
    l.P = l.b3 + dout;
    l.w2t = (uint64_t)din * H + (uint64_t)H * H + (uint64_t)H * dout;
    l.W = l.w2t + (uint64_t)H * H;
    return l;
}

// Adam (Kingma and Ba 2015, algorithm 1) on the fp32 parameters; weights also refresh their
// bfloat16 copies.  c1 = 1 - beta1^t, c2 = 1 - beta2^t.
__global__ void adam_step(float *p, const float *g, float *m, float *v, uint16_t *wb, Layout l, float lr,
                          float beta1, float beta2, float eps, float c1, float c2, int update)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < l.P; i += (uint64_t)gridDim.x * blockDim.x) {
        float pi = p[i];
        if (update) {
            const float gi = g[i];
            const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
            const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
            m[i] = mi;
            v[i] = vi;
            pi -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
            p[i] = pi;
        }
        int64_t w = -1;  // index in the bf16 copies
        if (i < l.b1) w = (int64_t)i;
        else if (i >= l.w2 && i < l.b2) w = (int64_t)(l.b1 + (i - l.w2));
        else if (i >= l.w3 && i < l.b3) w = (int64_t)(l.b1 + (l.b2 - l.w2) + (i - l.w3));
        if (w >= 0) wb[w] = f2bf(pi);
        if (i >= l.w2 && i < l.b2) {  // W2[k][n] -> W2T[n][k]
            const uint64_t H = l.w3 - l.b2;
            const uint64_t k = (i - l.w2) / H, n = (i - l.w2) % H;
            wb[l.w2t + n * H + k] = f2bf(pi);
        }
    }
}

// Inference of the whole network for kPredRows rows per workgroup (four waves), in one launch.
// The input tile and both hidden activations stay in LDS (bf16, rows padded by 8 elements);
// the layer products use the same MFMA tiles, k order and rounding points as mlp_gemm, so the
// outputs equal cae_mlp_forward's bit for bit.
constexpr uint32_t kPredRows = 32;
constexpr uint32_t kPredPad = 8;
constexpr uint32_t kPredMaxH = 496;  // keeps the workgroup's LDS within 64 KiB

struct PredArgs {
    const float *x;
    float *y;
    uint32_t N, din, H, dout;
    const uint16_t *W1, *W2T, *W3;
    const float *b1, *b2, *b3;
};

__device__ __forceinline__ v4s lds_frag(const uint16_t *p)  // four consecutive bf16
{
    const uint2 v = *reinterpret_cast<const uint2 *>(p);
    v4s r;
    r[0] = (short)(v.x & 0xFFFFu);
    r[1] = (short)(v.x >> 16);
    r[2] = (short)(v.y & 0xFFFFu);
    r[3] = (short)(v.y >> 16);
    return r;
}

__global__ void __launch_bounds__(256) mlp_predict(const PredArgs a)
{
    extern __shared__ __align__(16) uint16_t plds[];
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const uint32_t r16 = lane & 15u, grp = lane >> 4;
    const uint32_t row0 = blockIdx.x * kPredRows;
    const uint32_t Kx = (a.din + 15u) & ~15u;  // input width padded to the MFMA depth
    const uint32_t ldh = a.H + kPredPad;
    uint16_t *xs = plds;                        // [kPredRows][Kx]
    uint16_t *h1 = xs + kPredRows * Kx;          // [kPredRows][ldh]
    uint16_t *h2 = h1 + kPredRows * ldh;         // [kPredRows][ldh]
    for (uint32_t i = threadIdx.x; i < kPredRows * Kx; i += 256u) {
        const uint32_t r = i / Kx, c = i % Kx;
        xs[i] = (row0 + r < a.N && c < a.din) ? f2bf(a.x[(size_t)(row0 + r) * a.din + c]) : (uint16_t)0;
    }
    __syncthreads();
    const uint32_t ct = a.H / 16u;  // column tiles of a hidden layer
    // layer 1: h1 = silu(x W1 + b1)
    for (uint32_t j = wave; j < ct; j += 4u) {
        const uint32_t n = 16u * j + r16;
#pragma unroll
        for (uint32_t rt = 0; rt < kPredRows / 16u; ++rt) {
            v4f acc = {0.f, 0.f, 0.f, 0.f};
            for (uint32_t k0 = 0; k0 < Kx; k0 += 16u) {
                const v4s av = lds_frag(xs + (16u * rt + r16) * Kx + k0 + 4u * grp);
                v4s bv;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const uint32_t k = k0 + 4u * grp + (uint32_t)t;
                    bv[t] = (short)(k < a.din ? a.W1[(size_t)k * a.H + n] : (uint16_t)0);
                }
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const float z = acc[t] + a.b1[n];
                h1[(16u * rt + 4u * grp + (uint32_t)t) * ldh + n] = f2bf(silu(z));
            }
        }
    }
    __syncthreads();
    // layer 2: h2 = silu(h1 W2 + b2), B fragments from W2T (8 bytes per lane)
    for (uint32_t j = wave; j < ct; j += 4u) {
        const uint32_t n = 16u * j + r16;
        v4f acc[kPredRows / 16u];
#pragma unroll
        for (uint32_t rt = 0; rt < kPredRows / 16u; ++rt) acc[rt] = v4f{0.f, 0.f, 0.f, 0.f};
        const uint16_t *wrow = a.W2T + (size_t)n * a.H + 4u * grp;
        for (uint32_t k0 = 0; k0 < a.H; k0 += 128u) {
            v4s bv[8];
#pragma unroll
            for (uint32_t u = 0; u < 8u; ++u)
                if (k0 + 16u * u < a.H) {
                    const uint2 v = *reinterpret_cast<const uint2 *>(wrow + k0 + 16u * u);
                    bv[u][0] = (short)(v.x & 0xFFFFu);
                    bv[u][1] = (short)(v.x >> 16);
                    bv[u][2] = (short)(v.y & 0xFFFFu);
                    bv[u][3] = (short)(v.y >> 16);
                }
#pragma unroll
            for (uint32_t u = 0; u < 8u; ++u)
                if (k0 + 16u * u < a.H) {
#pragma unroll
                    for (uint32_t rt = 0; rt < kPredRows / 16u; ++rt) {
                        const v4s av = lds_frag(h1 + (16u * rt + r16) * ldh + k0 + 16u * u + 4u * grp);
                        acc[rt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv[u], acc[rt], 0, 0, 0);
                    }
                }
        }
#pragma unroll
        for (uint32_t rt = 0; rt < kPredRows / 16u; ++rt)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const float z = acc[rt][t] + a.b2[n];
                h2[(16u * rt + 4u * grp + (uint32_t)t) * ldh + n] = f2bf(silu(z));
            }
    }
    __syncthreads();
    // layer 3: y = h2 W3 + b3 (one column tile, one row tile per wave)
    if (wave < kPredRows / 16u) {
        const uint32_t rt = wave, n = r16;
        v4f acc = {0.f, 0.f, 0.f, 0.f};
        for (uint32_t k0 = 0; k0 < a.H; k0 += 16u) {
            const v4s av = lds_frag(h2 + (16u * rt + r16) * ldh + k0 + 4u * grp);
            v4s bv;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const uint32_t k = k0 + 4u * grp + (uint32_t)t;
                bv[t] = (short)(n < a.dout ? a.W3[(size_t)k * a.dout + n] : (uint16_t)0);
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
        }
        if (n < a.dout) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const uint32_t r = row0 + 16u * rt + 4u * grp + (uint32_t)t;
                if (r < a.N) a.y[(size_t)r * a.dout + n] = acc[t] + a.b3[n];
            }
        }
    }
}

// ------------------------------------------------------------------------------------------
// Fused training step: forward, loss gradient, back-propagation and Adam in two launches, on
// gfx950's v_mfma_f32_16x16x32_bf16 (eight bfloat16 of the reduction per lane and operand).
//
// mlp_train_rows: one workgroup per 16 batch rows.  The rows' input, both hidden activations,
//   their pre-activations, the loss gradient and the first back-propagated gradient stay in LDS;
//   every operand fragment is one 16-byte read (LDS rows, the bfloat16 W2 and its transposed
//   copy).  The activations and gradients the weight gradients need are written to the
//   workspace transposed ([feature][batch], 8-byte stores), so that the next kernel reads its
//   fragments (eight consecutive batch rows) with 16-byte loads as well.
// mlp_train_params: one wave per 16x16 tile of a weight gradient (with the bias as the extra row
//   of ones, as in the unfused path), reduced over the whole batch in a fixed order by the wave
//   that owns it -- no split-K partials, deterministic -- followed in the same wave by Adam and
//   the bfloat16 copies of the updated weights.
// Rounding points and fp32 accumulation are those of the unfused kernels; only the order of the
// fp32 sums differs.
// ------------------------------------------------------------------------------------------
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr uint32_t kTrainRows = 16;
constexpr uint32_t kRowWaves = 16;   // waves of an mlp_train_rows workgroup: one 16-column tile each at H = 256
constexpr uint32_t kParamSplit = 4;  // waves that reduce one weight-gradient tile, each a quarter of the batch
// reduction steps whose global operand loads are issued together before their matrix-core chain
// (the chain's order, and so every rounding, is the step-by-step one)
constexpr uint32_t kLoadAhead = 8;
constexpr uint32_t kTrainMaxH = 256;
constexpr uint32_t kTrainMaxIn = 32;
constexpr uint32_t kTrainPad = 8;  // bf16 elements of padding per LDS row

__device__ __forceinline__ v8bf ld8(const uint16_t *p)  // eight bfloat16, 16-byte aligned
{
    return __builtin_bit_cast(v8bf, *reinterpret_cast<const uint4 *>(p));
}

__device__ __forceinline__ v8bf pack8(const uint16_t (&e)[8])
{
    uint4 u;
    u.x = (uint32_t)e[0] | ((uint32_t)e[1] << 16);
    u.y = (uint32_t)e[2] | ((uint32_t)e[3] << 16);
    u.z = (uint32_t)e[4] | ((uint32_t)e[5] << 16);
    u.w = (uint32_t)e[6] | ((uint32_t)e[7] << 16);
    return __builtin_bit_cast(v8bf, u);
}

__device__ __forceinline__ v4f mfma32(v8bf a, v8bf b, v4f c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// four bfloat16 of consecutive batch rows into a transposed [feature][batch] array
__device__ __forceinline__ void st4(uint16_t *p, uint16_t a, uint16_t b, uint16_t c, uint16_t d)
{
    *reinterpret_cast<uint2 *>(p) = make_uint2((uint32_t)a | ((uint32_t)b << 16), (uint32_t)c | ((uint32_t)d << 16));
}

struct TrainArgs {
    const float *x, *t;      // all samples: x[n][din], t[n][dout]
    const uint32_t *idx;     // the batch's sample indices (NULL: 0..B-1)
    uint32_t B, Bp;          // batch, and batch rounded up to 32 (leading dim of the T arrays)
    uint32_t din, H, dout;
    const uint16_t *W1, *W2, *W2T, *W3;
    float *p, *m, *v, *grads;  // fp32 parameters, Adam moments, optional gradient output
    uint16_t *wb;              // bfloat16 weight copies
    uint16_t *xT, *h1T, *h2T, *dyT, *dz2T, *dz1T;
    float *loss_part, *loss;
    Layout l;
    int kind;
    float delta, inv_n;        // Huber delta; 1 / (B dout)
    float lr, beta1, beta2, eps, c1, c2;
    uint32_t tiles1, tiles2, tiles3;  // gradient tiles of W1|b1, W2|b2, W3|b3
};

// Every operand that does not depend on the rows (the wave's weight fragments and biases, and
// wave 0's targets) is loaded before the phase that precedes its use, so that each phase's
// memory latency overlaps the one before instead of following a barrier; W3, which layer 3
// gathers column by column, is copied to LDS at the start.  At H <= 256 a wave owns
// one 16-column tile and a reduction over H is at most kLoadAhead matrix-core steps.
static_assert(kTrainMaxH <= 16u * kRowWaves && kTrainMaxH <= 32u * kLoadAhead, "one tile per wave, one load chunk");

__global__ void __launch_bounds__(kRowWaves * 64) mlp_train_rows(const TrainArgs a)
{
    extern __shared__ __align__(16) unsigned char tlds[];
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const uint32_t r = lane & 15u, g = lane >> 4;
    const uint32_t row0 = blockIdx.x * kTrainRows;
    const uint32_t H = a.H, ldh = H + kTrainPad, ct = H / 16u;
    uint16_t *xs = reinterpret_cast<uint16_t *>(tlds);  // [16][32]
    uint16_t *dys = xs + kTrainRows * 32u;               // [16][32]
    uint16_t *h1s = dys + kTrainRows * 32u;              // [16][ldh]
    uint16_t *h2s = h1s + kTrainRows * ldh;
    uint16_t *dzs = h2s + kTrainRows * ldh;
    float *z1s = reinterpret_cast<float *>(dzs + kTrainRows * ldh);  // [16][H]
    float *z2s = z1s + kTrainRows * H;
    uint16_t *w3s = reinterpret_cast<uint16_t *>(z2s + kTrainRows * H);  // W3 [H][d_out]
    const bool tile = wave < ct;  // the wave's output columns n = 16 wave + (lane % 16)
    const uint32_t n = 16u * wave + r;
    // W3 (at most 256 x 16) for layer 3 and the dz2 step, copied to LDS by the whole workgroup
    for (uint32_t i = threadIdx.x; i < H * a.dout; i += kRowWaves * 64u) w3s[i] = a.W3[i];
    // the wave's operands of layer 1 (W1 column n) and layer 2 (W2T row n), and both biases
    uint16_t e1[8];
    v8bf w2t[kLoadAhead];
    float b1n = 0.f, b2n = 0.f;
    if (tile) {
#pragma unroll
        for (uint32_t t = 0; t < 8u; ++t) {
            const uint32_t k = 8u * g + t;
            e1[t] = k < a.din ? a.W1[(size_t)k * H + n] : (uint16_t)0;
        }
#pragma unroll
        for (uint32_t u = 0; u < kLoadAhead; ++u)
            if (32u * u < H) w2t[u] = ld8(a.W2T + (size_t)n * H + 32u * u + 8u * g);
        b1n = a.p[a.l.b1 + n];
        b2n = a.p[a.l.b2 + n];
    }
    // wave 0's layer-3 operands: b3 and the rows' targets (zero past the batch or d_out)
    float b3r = 0.f, tv[4] = {0.f, 0.f, 0.f, 0.f};
    if (wave == 0) {
        if (r < a.dout) b3r = a.p[a.l.b3 + r];
#pragma unroll
        for (uint32_t t = 0; t < 4u; ++t) {
            const uint32_t row = row0 + 4u * g + t;
            if (row < a.B && r < a.dout) {
                const uint32_t src = a.idx ? a.idx[row] : row;
                tv[t] = a.t[(size_t)src * a.dout + r];
            }
        }
    }
    // inputs of the rows (zero past the batch), their transposed copy, and a zeroed dy tile
    for (uint32_t i = threadIdx.x; i < kTrainRows * 32u; i += kRowWaves * 64u) {
        const uint32_t rr = i / 32u, c = i % 32u, row = row0 + rr;
        uint16_t v = 0;
        if (row < a.B && c < a.din) {
            const uint32_t src = a.idx ? a.idx[row] : row;
            v = f2bf(a.x[(size_t)src * a.din + c]);
        }
        xs[i] = v;
        dys[i] = 0;
        if (c < a.din) a.xT[(size_t)c * a.Bp + row] = v;
    }
    __syncthreads();
    // layer 1: z1 = x W1 + b1, h1 = silu(z1)  (one reduction step: d_in <= 32)
    if (tile) {
        v4f acc = {0.f, 0.f, 0.f, 0.f};
        acc = mfma32(ld8(xs + r * 32u + 8u * g), pack8(e1), acc);
        uint16_t hb[4];
#pragma unroll
        for (uint32_t t = 0; t < 4u; ++t) {
            const uint32_t rr = 4u * g + t;
            const float z = acc[t] + b1n;
            z1s[rr * H + n] = z;
            hb[t] = f2bf(silu(z));
            h1s[rr * ldh + n] = hb[t];
        }
        st4(a.h1T + (size_t)n * a.Bp + row0 + 4u * g, hb[0], hb[1], hb[2], hb[3]);
    }
    __syncthreads();
    // layer 2: z2 = h1 W2 + b2, B fragments from the transposed copy W2T[n][k]; then the W2
    // fragments of the dz1 step, in flight through layer 3 and the dz2 step
    v8bf w2[kLoadAhead];
    if (tile) {
        v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (uint32_t u = 0; u < kLoadAhead; ++u)
            if (32u * u < H) acc = mfma32(ld8(h1s + r * ldh + 32u * u + 8u * g), w2t[u], acc);
        uint16_t hb[4];
#pragma unroll
        for (uint32_t t = 0; t < 4u; ++t) {
            const uint32_t rr = 4u * g + t;
            const float z = acc[t] + b2n;
            z2s[rr * H + n] = z;
            hb[t] = f2bf(silu(z));
            h2s[rr * ldh + n] = hb[t];
        }
        st4(a.h2T + (size_t)n * a.Bp + row0 + 4u * g, hb[0], hb[1], hb[2], hb[3]);
#pragma unroll
        for (uint32_t u = 0; u < kLoadAhead; ++u)
            if (32u * u < H) w2[u] = ld8(a.W2 + (size_t)n * H + 32u * u + 8u * g);
    }
    __syncthreads();
    // layer 3, loss and its gradient (one wave): y = h2 W3 + b3; dy = dloss/dy, zero past the batch
    if (wave == 0) {
        v4f acc = {0.f, 0.f, 0.f, 0.f};
        for (uint32_t k0 = 0; k0 < H; k0 += 32u) {
            uint16_t e[8];  // W3 column r from LDS, zero past d_out
#pragma unroll
            for (uint32_t t = 0; t < 8u; ++t) e[t] = r < a.dout ? w3s[(k0 + 8u * g + t) * a.dout + r] : (uint16_t)0;
            acc = mfma32(ld8(h2s + r * ldh + k0 + 8u * g), pack8(e), acc);
        }
        float ls = 0.f;
        uint16_t db[4];
#pragma unroll
        for (uint32_t t = 0; t < 4u; ++t) {
            const uint32_t rr = 4u * g + t, row = row0 + rr;
            float dy = 0.f;
            if (row < a.B && r < a.dout) {
                const float d = acc[t] + b3r - tv[t];
                if (a.kind == CAE_LOSS_MSE) {
                    dy = 2.0f * d * a.inv_n;
                    ls += d * d;
                } else {
                    const float ad = fabsf(d);
                    dy = fminf(fmaxf(d, -a.delta), a.delta) * a.inv_n;
                    ls += ad <= a.delta ? 0.5f * d * d : a.delta * (ad - 0.5f * a.delta);
                }
            }
            db[t] = f2bf(dy);
            dys[rr * 32u + r] = db[t];
        }
        st4(a.dyT + (size_t)r * a.Bp + row0 + 4u * g, db[0], db[1], db[2], db[3]);
        // the rows' loss, summed over the wave in a fixed order
#pragma unroll
        for (uint32_t off = 32u; off > 0u; off >>= 1) ls += __shfl_xor(ls, (int)off);
        if (lane == 0) a.loss_part[blockIdx.x] = ls;
    }
    __syncthreads();
    // dz2 = (dy W3^T) silu'(z2)  (one reduction step: d_out <= 16)
    if (tile) {
        uint16_t e3[8];  // W3 row n from LDS, zero past d_out
#pragma unroll
        for (uint32_t t = 0; t < 8u; ++t) {
            const uint32_t k = 8u * g + t;
            e3[t] = k < a.dout ? w3s[n * a.dout + k] : (uint16_t)0;
        }
        v4f acc = {0.f, 0.f, 0.f, 0.f};
        acc = mfma32(ld8(dys + r * 32u + 8u * g), pack8(e3), acc);
        uint16_t zb[4];
#pragma unroll
        for (uint32_t t = 0; t < 4u; ++t) {
            const uint32_t rr = 4u * g + t;
            zb[t] = f2bf(acc[t] * dsilu(z2s[rr * H + n]));
            dzs[rr * ldh + n] = zb[t];
        }
        st4(a.dz2T + (size_t)n * a.Bp + row0 + 4u * g, zb[0], zb[1], zb[2], zb[3]);
    }
    __syncthreads();
    // dz1 = (dz2 W2^T) silu'(z1): B fragments W2[n][k], eight consecutive k
    if (tile) {
        v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (uint32_t u = 0; u < kLoadAhead; ++u)
            if (32u * u < H) acc = mfma32(ld8(dzs + r * ldh + 32u * u + 8u * g), w2[u], acc);
        uint16_t zb[4];
#pragma unroll
        for (uint32_t t = 0; t < 4u; ++t) zb[t] = f2bf(acc[t] * dsilu(z1s[(4u * g + t) * H + n]));
        st4(a.dz1T + (size_t)n * a.Bp + row0 + 4u * g, zb[0], zb[1], zb[2], zb[3]);
    }
}

// One Adam update of parameter i with gradient gi (Kingma and Ba 2015, algorithm 1).
__device__ __forceinline__ float adam_one(const TrainArgs &a, uint64_t i, float gi)
{
    const float mi = a.beta1 * a.m[i] + (1.0f - a.beta1) * gi;
    const float vi = a.beta2 * a.v[i] + (1.0f - a.beta2) * gi * gi;
    a.m[i] = mi;
    a.v[i] = vi;
    const float pi = a.p[i] - a.lr * (mi / a.c1) / (sqrtf(vi / a.c2) + a.eps);
    a.p[i] = pi;
    if (a.grads) a.grads[i] = gi;
    return pi;
}

__global__ void __launch_bounds__(kParamSplit * 64) mlp_train_params(const TrainArgs a)
{
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const uint32_t r = lane & 15u, g = lane >> 4;
    if (blockIdx.x == 0 && threadIdx.x == 0) {  // mean loss of the batch, partials in row order
        float s = 0.f;
        for (uint32_t i = 0; i < a.Bp / kTrainRows; ++i) s += a.loss_part[i];
        a.loss[0] = s * a.inv_n;
    }
    uint32_t tile = blockIdx.x;  // kParamSplit waves per tile
    const uint32_t H = a.H, din = a.din, dout = a.dout, ct = H / 16u;
    // which gradient: [A^T ; 1] B over the batch, A the layer's input, B its output gradient
    const uint16_t *AT, *BT;
    uint32_t M, N, ti, tj;
    uint64_t woff, boff, wcopy;
    if (tile < a.tiles1) {
        AT = a.xT, BT = a.dz1T, M = din, N = H, ti = tile / ct, tj = tile % ct;
        woff = a.l.w1, boff = a.l.b1, wcopy = 0;
    } else if ((tile -= a.tiles1) < a.tiles2) {
        AT = a.h1T, BT = a.dz2T, M = H, N = H, ti = tile / ct, tj = tile % ct;
        woff = a.l.w2, boff = a.l.b2, wcopy = (uint64_t)din * H;
    } else if ((tile -= a.tiles2) < a.tiles3) {
        AT = a.h2T, BT = a.dyT, M = H, N = dout, ti = tile, tj = 0;
        woff = a.l.w3, boff = a.l.b3, wcopy = (uint64_t)din * H + (uint64_t)H * H;
    } else {
        return;
    }
    const uint32_t i = ti * 16u + r, j = tj * 16u + r;  // A row and B column this lane feeds
    v8bf ones;
#pragma unroll
    for (int t = 0; t < 8; ++t) ones[t] = (__bf16)1.0f;
    v8bf zero;
#pragma unroll
    for (int t = 0; t < 8; ++t) zero[t] = (__bf16)0.0f;
    const bool arow = i < M, brow = j < N;  // rows >= Bp of the transposed arrays do not exist
    const uint16_t *ap = AT + (size_t)(arow ? i : 0) * a.Bp + 8u * g;
    const uint16_t *bp = BT + (size_t)(brow ? j : 0) * a.Bp + 8u * g;
    // wave w reduces the batch chunks w, w + kParamSplit, ... of 32 rows; the partial sums are
    // then added in wave order (a fixed order: deterministic)
    __shared__ v4f part[kParamSplit][64];
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    for (uint32_t c0 = 32u * wave; c0 < a.Bp; c0 += 32u * kParamSplit * kLoadAhead) {
        v8bf av[kLoadAhead], bv[kLoadAhead];  // the chunk's fragments, in flight together
#pragma unroll
        for (uint32_t u = 0; u < kLoadAhead; ++u) {
            const uint32_t b0 = c0 + 32u * kParamSplit * u;
            if (b0 < a.Bp) {
                av[u] = arow ? ld8(ap + b0) : (i == M ? ones : zero);
                bv[u] = brow ? ld8(bp + b0) : zero;
            }
        }
#pragma unroll
        for (uint32_t u = 0; u < kLoadAhead; ++u)
            if (c0 + 32u * kParamSplit * u < a.Bp) acc = mfma32(av[u], bv[u], acc);
    }
    part[wave][lane] = acc;
    __syncthreads();
    if (wave != 0u) return;
    acc = part[0][lane];
#pragma unroll
    for (uint32_t w = 1; w < kParamSplit; ++w) acc += part[w][lane];
    const uint32_t jc = tj * 16u + r;
    if (jc >= N) return;
#pragma unroll
    for (uint32_t t = 0; t < 4u; ++t) {
        const uint32_t ic = ti * 16u + 4u * g + t;
        if (ic > M) continue;
        if (ic == M) {
            adam_one(a, boff + jc, acc[t]);
        } else {
            const float pi = adam_one(a, woff + (uint64_t)ic * N + jc, acc[t]);
            const uint16_t w = f2bf(pi);
            a.wb[wcopy + (uint64_t)ic * N + jc] = w;
            if (woff == a.l.w2) a.wb[a.l.w2t + (uint64_t)jc * H + ic] = w;
        }
    }
}

}  // namespace

namespace {
int forward_impl(const cae_mlp *net, const float *x, float *y, uint32_t N, void *ws, hipStream_t s);
}  // namespace

namespace cae_detail {
int set_error(int code, const char *msg);  // cae_engine.hip: message for cae_last_error()
}

namespace {

int mfail(int code, const char *msg) { return cae_detail::set_error(code, msg); }

struct WsLayout {
    size_t xb, z1, h1, z2, h2, dyb, dz2, dz1, part, total;
};

constexpr uint32_t kSplitChunk = 256;  // batch rows per split-K part of a weight gradient
constexpr uint32_t kMaxParts = 64;

size_t al(size_t x) { return (x + 255) / 256 * 256; }

WsLayout ws_layout(uint32_t din, uint32_t H, uint32_t dout, uint32_t N)
{
    WsLayout w;
    size_t o = 0;
    w.xb = o; o = al(o + 2ull * N * din);
    w.z1 = o; o = al(o + 4ull * N * H);
    w.h1 = o; o = al(o + 2ull * N * H);
    w.z2 = o; o = al(o + 4ull * N * H);
    w.h2 = o; o = al(o + 2ull * N * H);
    w.dyb = o; o = al(o + 2ull * N * dout);
    w.dz2 = o; o = al(o + 2ull * N * H);
    w.dz1 = o; o = al(o + 2ull * N * H);
    const uint64_t parts = std::min<uint64_t>(kMaxParts, (N + kSplitChunk - 1) / kSplitChunk);
    const uint64_t rows = std::max<uint64_t>(din, H) + 1;
    w.part = o; o = al(o + 4ull * parts * rows * std::max<uint32_t>(H, dout));
    w.total = o;
    return w;
}

// Workspace of the fused training step: the transposed activations and gradients ([rows][Bp]
// bfloat16, Bp = the batch rounded up to 32) and one loss partial per 16 rows.
struct TrainWs {
    size_t xT, h1T, h2T, dyT, dz2T, dz1T, loss_part, total;
};

TrainWs train_ws(uint32_t din, uint32_t H, uint32_t N)
{
    const size_t Bp = (N + 31u) / 32u * 32u;
    TrainWs w;
    size_t o = 0;
    w.xT = o; o = al(o + 2 * din * Bp);
    w.h1T = o; o = al(o + 2 * (size_t)H * Bp);
    w.h2T = o; o = al(o + 2 * (size_t)H * Bp);
    w.dyT = o; o = al(o + 2 * 16 * Bp);
    w.dz2T = o; o = al(o + 2 * (size_t)H * Bp);
    w.dz1T = o; o = al(o + 2 * (size_t)H * Bp);
    w.loss_part = o; o = al(o + 4 * (Bp / kTrainRows));
    w.total = o;
    return w;
}

int check_net(const cae_mlp *net)
{
    if (!net || !net->params || !net->weights) return mfail(CAE_EINVAL, "NULL network or buffer");
    if (net->d_in < 1 || net->d_in > 64) return mfail(CAE_EINVAL, "d_in must be in 1..64");
    if (net->d_hidden < 16 || net->d_hidden > 1024 || net->d_hidden % 16)
        return mfail(CAE_EINVAL, "d_hidden must be a multiple of 16 in 16..1024");
    if (net->d_out < 1 || net->d_out > 16) return mfail(CAE_EINVAL, "d_out must be in 1..16");
    return CAE_OK;
}

template <bool TA, bool TB, int EPI>
void gemm(GemmArgs g, hipStream_t s)
{
    if (g.kchunk == 0) g.kchunk = g.K;
    const uint32_t tiles = ((g.M + g.ones_row + 15u) / 16u) * ((g.N + 15u) / 16u);
    hipLaunchKernelGGL((mlp_gemm<TA, TB, EPI>), dim3((tiles + 3u) / 4u), dim3(256), 0, s, g);
}

// Weight gradient [M+1][N] = [A^T ; 1^T] B over the batch (the last row is the bias gradient),
// split over batch chunks into partials and summed in chunk order.
void weight_grad(const uint16_t *A, uint32_t lda, const uint16_t *B, uint32_t ldb, uint32_t M, uint32_t N,
                 uint32_t batch, float *out, float *part, hipStream_t s)
{
    GemmArgs g{};
    g.A = A;
    g.B = B;
    g.lda = lda;
    g.ldb = ldb;
    g.M = M;
    g.N = N;
    g.K = batch;
    g.ones_row = 1;
    g.ldo = N;
    const uint32_t parts = std::min<uint32_t>(kMaxParts, (batch + kSplitChunk - 1) / kSplitChunk);
    g.kchunk = ((batch + parts - 1) / parts + 15u) / 16u * 16u;
    const uint32_t nparts = (batch + g.kchunk - 1) / g.kchunk;
    g.Of = nparts > 1 ? part : out;
    const uint32_t tiles = ((M + 1 + 15u) / 16u) * ((N + 15u) / 16u);
    hipLaunchKernelGGL((mlp_gemm<true, false, EPI_F32>), dim3((tiles + 3u) / 4u, nparts), dim3(256), 0, s, g);
    if (nparts > 1) {
        const uint64_t n = (uint64_t)(M + 1) * N;
        hipLaunchKernelGGL(sum_partials, dim3((uint32_t)std::min<uint64_t>((n + 255) / 256, 1024)), dim3(256), 0, s,
                           part, nparts, n, out);
    }
}

GemmArgs gargs(const uint16_t *A, uint32_t lda, const uint16_t *B, uint32_t ldb, uint32_t M, uint32_t N, uint32_t K)
{
    GemmArgs g{};
    g.A = A;
    g.B = B;
    g.lda = lda;
    g.ldb = ldb;
    g.M = M;
    g.N = N;
    g.K = K;
    return g;
}

int launch_status()
{
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return mfail(CAE_EHIP, hipGetErrorString(e));
    return CAE_OK;
}

// Scratch of cae_mlp_train_step_noalloc: the fused training step's workspace (transposed
// activations and gradients, loss partials) for callers that cannot allocate device memory.
// Every device the library runs on holds its own copy until the process ends; host code must not
// pass the array's name to a kernel (it is a host-side stand-in), only the per-device address
// that hipGetSymbolAddress returns.  Nothing in it needs clearing between calls: each call's
// first kernel writes every word its second kernel reads.
constexpr size_t kScratchBytes = size_t(8) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The address of the current device's copy of `scratch`, looked up once per device.
int scratch_of_current_device(void **out)
{
    int dev = -1;
    hipError_t he = hipGetDevice(&dev);
    if (he != hipSuccess) return mfail(CAE_EHIP, hipGetErrorString(he));
    if (dev < 0 || dev >= kMaxDevices) return mfail(CAE_EINVAL, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        he = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (he != hipSuccess || !p)
            return mfail(CAE_EHIP, he != hipSuccess ? hipGetErrorString(he) : "no address for the scratch array");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return CAE_OK;
}

// Argument checks shared by both training-step entry points (no device call).
int check_train_args(const cae_mlp *net, const float *x, const float *target, const float *m, const float *v,
                     uint32_t N, uint32_t step, int loss_kind, float delta, const float *loss)
{
    int rc = check_net(net);
    if (rc) return rc;
    const uint32_t din = net->d_in, H = net->d_hidden;
    if (H % 32u || H > kTrainMaxH || din > kTrainMaxIn)
        return mfail(CAE_EINVAL, "cae_mlp_train_step needs d_hidden a multiple of 32 up to 256 and d_in <= 32");
    if (!x || !target || !m || !v || !loss) return mfail(CAE_EINVAL, "NULL pointer");
    if (N == 0) return mfail(CAE_EINVAL, "N must be >= 1");
    if (step < 1) return mfail(CAE_EINVAL, "step counts from 1");
    if (loss_kind != CAE_LOSS_MSE && loss_kind != CAE_LOSS_HUBER) return mfail(CAE_EINVAL, "unknown loss kind");
    if (loss_kind == CAE_LOSS_HUBER && !(delta > 0.0f)) return mfail(CAE_EINVAL, "Huber delta must be > 0");
    return CAE_OK;
}

// The fused training step (two launches) on a workspace of train_ws(d_in, H, N).total bytes.
int train_step_impl(const cae_mlp *net, const float *x, const float *target, const uint32_t *idx, uint32_t N,
                    float *m, float *v, uint32_t step, float lr, float beta1, float beta2, float eps, int loss_kind,
                    float delta, float *loss, float *grads, void *ws, hipStream_t s)
{
    const uint32_t din = net->d_in, H = net->d_hidden, dout = net->d_out;
    const Layout l = layout(din, H, dout);
    const TrainWs w = train_ws(din, H, N);
    unsigned char *b = static_cast<unsigned char *>(ws);
    TrainArgs a;
    a.x = x;
    a.t = target;
    a.idx = idx;
    a.B = N;
    a.Bp = (N + 31u) / 32u * 32u;
    a.din = din;
    a.H = H;
    a.dout = dout;
    a.W1 = net->weights;
    a.W2 = a.W1 + (size_t)din * H;
    a.W3 = a.W2 + (size_t)H * H;
    a.W2T = net->weights + l.w2t;
    a.p = net->params;
    a.m = m;
    a.v = v;
    a.grads = grads;
    a.wb = net->weights;
    a.xT = reinterpret_cast<uint16_t *>(b + w.xT);
    a.h1T = reinterpret_cast<uint16_t *>(b + w.h1T);
    a.h2T = reinterpret_cast<uint16_t *>(b + w.h2T);
    a.dyT = reinterpret_cast<uint16_t *>(b + w.dyT);
    a.dz2T = reinterpret_cast<uint16_t *>(b + w.dz2T);
    a.dz1T = reinterpret_cast<uint16_t *>(b + w.dz1T);
    a.loss_part = reinterpret_cast<float *>(b + w.loss_part);
    a.loss = loss;
    a.l = l;
    a.kind = loss_kind;
    a.delta = delta;
    a.inv_n = 1.0f / (float)((double)N * dout);
    a.lr = lr;
    a.beta1 = beta1;
    a.beta2 = beta2;
    a.eps = eps;
    a.c1 = (float)(1.0 - std::pow((double)beta1, (double)step));
    a.c2 = (float)(1.0 - std::pow((double)beta2, (double)step));
    const uint32_t ct = H / 16u;
    a.tiles1 = (din + 1u + 15u) / 16u * ct;
    a.tiles2 = (H / 16u + 1u) * ct;
    a.tiles3 = H / 16u + 1u;
    const size_t lds = 2ull * (2u * kTrainRows * 32u + 3ull * kTrainRows * (H + kTrainPad)) + 8ull * kTrainRows * H +
                       2ull * H * dout;  // + W3 in bf16
    hipLaunchKernelGGL(mlp_train_rows, dim3(a.Bp / kTrainRows), dim3(kRowWaves * 64u), lds, s, a);
    const uint32_t tiles = a.tiles1 + a.tiles2 + a.tiles3;
    hipLaunchKernelGGL(mlp_train_params, dim3(tiles), dim3(kParamSplit * 64u), 0, s, a);
    return launch_status();
}

}  // namespace

extern "C" {

int cae_mlp_sizes(uint32_t d_in, uint32_t d_hidden, uint32_t d_out, uint32_t max_batch, cae_mlp_sizes_t *out)
{
    if (!out) return mfail(CAE_EINVAL, "out is NULL");
    cae_mlp probe{d_in, d_hidden, d_out, 0, reinterpret_cast<float *>(1), reinterpret_cast<uint16_t *>(1)};
    int rc = check_net(&probe);
    if (rc) return rc;
    const Layout l = layout(d_in, d_hidden, d_out);
    out->n_params = l.P;
    out->n_weights = l.W;
    out->workspace_bytes = std::max(ws_layout(d_in, d_hidden, d_out, max_batch).total,
                                    train_ws(d_in, d_hidden, max_batch).total);
    return CAE_OK;
}

int cae_mlp_refresh_weights(const cae_mlp *net, void *stream)
{
    int rc = check_net(net);
    if (rc) return rc;
    const Layout l = layout(net->d_in, net->d_hidden, net->d_out);
    hipLaunchKernelGGL(adam_step, dim3(256), dim3(256), 0, (hipStream_t)stream, net->params, nullptr, nullptr,
                       nullptr, net->weights, l, 0.f, 0.f, 0.f, 0.f, 1.f, 1.f, 0);
    return launch_status();
}

int cae_mlp_forward(const cae_mlp *net, const float *x, float *y, uint32_t N, void *ws, void *stream)
{
    int rc = check_net(net);
    if (rc) return rc;
    if (!x || !y || !ws) return mfail(CAE_EINVAL, "NULL x, y or workspace");
    if (N == 0) return CAE_OK;
    return forward_impl(net, x, y, N, ws, (hipStream_t)stream);
}

int cae_mlp_predict(const cae_mlp *net, const float *x, float *y, uint32_t N, void *stream)
{
    int rc = check_net(net);
    if (rc) return rc;
    if (!x || !y) return mfail(CAE_EINVAL, "NULL x or y");
    if (net->d_hidden > kPredMaxH) return mfail(CAE_EINVAL, "cae_mlp_predict needs d_hidden <= 496");
    if (N == 0) return CAE_OK;
    const uint32_t din = net->d_in, H = net->d_hidden, dout = net->d_out;
    const Layout l = layout(din, H, dout);
    PredArgs a;
    a.x = x;
    a.y = y;
    a.N = N;
    a.din = din;
    a.H = H;
    a.dout = dout;
    a.W1 = net->weights;
    a.W2T = net->weights + l.w2t;
    a.W3 = net->weights + (size_t)din * H + (size_t)H * H;
    a.b1 = net->params + l.b1;
    a.b2 = net->params + l.b2;
    a.b3 = net->params + l.b3;
    const size_t lds = 2ull * (kPredRows * ((din + 15u) & ~15u) + 2ull * kPredRows * (H + kPredPad));
    const uint32_t blocks = (N + kPredRows - 1u) / kPredRows;
    hipLaunchKernelGGL(mlp_predict, dim3(blocks), dim3(256), lds, (hipStream_t)stream, a);
    return launch_status();
}

int cae_mlp_backward(const cae_mlp *net, const float *x, const float *dy, float *grads, uint32_t N, void *ws,
                     void *stream)
{
    (void)x;  // the bfloat16 input is taken from the forward pass's workspace
    int rc = check_net(net);
    if (rc) return rc;
    if (!dy || !grads || !ws) return mfail(CAE_EINVAL, "NULL dy, grads or workspace");
    hipStream_t s = (hipStream_t)stream;
    const uint32_t din = net->d_in, H = net->d_hidden, dout = net->d_out;
    const Layout l = layout(din, H, dout);
    const WsLayout w = ws_layout(din, H, dout, N);
    unsigned char *b = static_cast<unsigned char *>(ws);
    const uint16_t *xb = reinterpret_cast<const uint16_t *>(b + w.xb);
    const float *z1 = reinterpret_cast<const float *>(b + w.z1);
    const uint16_t *h1 = reinterpret_cast<const uint16_t *>(b + w.h1);
    const float *z2 = reinterpret_cast<const float *>(b + w.z2);
    const uint16_t *h2 = reinterpret_cast<const uint16_t *>(b + w.h2);
    uint16_t *dyb = reinterpret_cast<uint16_t *>(b + w.dyb);
    uint16_t *dz2 = reinterpret_cast<uint16_t *>(b + w.dz2);
    uint16_t *dz1 = reinterpret_cast<uint16_t *>(b + w.dz1);
    float *part = reinterpret_cast<float *>(b + w.part);
    const uint16_t *W1 = net->weights, *W2 = W1 + (size_t)din * H, *W3 = W2 + (size_t)H * H;
    (void)W1;
    if (N == 0) return mfail(CAE_EINVAL, "backward needs N >= 1");
    const uint64_t ny = (uint64_t)N * dout;
    hipLaunchKernelGGL(to_bf16, dim3((uint32_t)std::min<uint64_t>((ny + 255) / 256, 1024)), dim3(256), 0, s, dy, dyb, ny);
    // output layer: [dW3; db3] = [h2; 1]^T dy (b3 directly follows W3 in the layout)
    weight_grad(h2, H, dyb, dout, H, dout, N, grads + l.w3, part, s);
    // dz2 = (dy W3^T) * silu'(z2)
    GemmArgs g = gargs(dyb, dout, W3, dout, N, H, dout);
    g.Zin = z2;
    g.Ob = dz2;
    g.ldo = H;
    gemm<false, true, EPI_DSILU>(g, s);
    weight_grad(h1, H, dz2, H, H, H, N, grads + l.w2, part, s);
    // dz1 = (dz2 W2^T) * silu'(z1)
    g = gargs(dz2, H, W2, H, N, H, H);
    g.Zin = z1;
    g.Ob = dz1;
    g.ldo = H;
    gemm<false, true, EPI_DSILU>(g, s);
    weight_grad(xb, din, dz1, H, din, H, N, grads + l.w1, part, s);
    return launch_status();
}

int cae_mlp_adam(const cae_mlp *net, const float *grads, float *m, float *v, uint32_t step, float lr, float beta1,
                 float beta2, float eps, void *stream)
{
    int rc = check_net(net);
    if (rc) return rc;
    if (!grads || !m || !v) return mfail(CAE_EINVAL, "NULL grads or moments");
    if (step < 1) return mfail(CAE_EINVAL, "step counts from 1");
    const Layout l = layout(net->d_in, net->d_hidden, net->d_out);
    const float c1 = (float)(1.0 - std::pow((double)beta1, (double)step));
    const float c2 = (float)(1.0 - std::pow((double)beta2, (double)step));
    hipLaunchKernelGGL(adam_step, dim3((uint32_t)std::min<uint64_t>((l.P + 255) / 256, 1024)), dim3(256), 0,
                       (hipStream_t)stream, net->params, grads, m, v, net->weights, l, lr, beta1, beta2, eps, c1, c2, 1);
    return launch_status();
}

int cae_mlp_train_step(const cae_mlp *net, const float *x, const float *target, const uint32_t *idx, uint32_t N,
                       float *m, float *v, uint32_t step, float lr, float beta1, float beta2, float eps, int loss_kind,
                       float delta, float *loss, float *grads, void *ws, void *stream)
{
    int rc = check_train_args(net, x, target, m, v, N, step, loss_kind, delta, loss);
    if (rc) return rc;
    if (!ws) return mfail(CAE_EINVAL, "NULL workspace");
    return train_step_impl(net, x, target, idx, N, m, v, step, lr, beta1, beta2, eps, loss_kind, delta, loss, grads,
                           ws, (hipStream_t)stream);
}

int cae_mlp_train_step_noalloc(const cae_mlp *net, const float *x, const float *target, const uint32_t *idx,
                               uint32_t N, float *m, float *v, uint32_t step, float lr, float beta1, float beta2,
                               float eps, int loss_kind, float delta, float *loss, float *grads, void *stream)
{
    int rc = check_train_args(net, x, target, m, v, N, step, loss_kind, delta, loss);
    if (rc) return rc;
    const size_t need = train_ws(net->d_in, net->d_hidden, N).total;
    if (need > kScratchBytes) {
        char msg[160];
        std::snprintf(msg, sizeof msg,
                      "cae_mlp_train_step_noalloc: batch %u needs %zu bytes of scratch, the library holds %zu", N,
                      need, kScratchBytes);
        return mfail(CAE_EINVAL, msg);
    }
    void *ws = nullptr;
    rc = scratch_of_current_device(&ws);
    if (rc) return rc;
    return train_step_impl(net, x, target, idx, N, m, v, step, lr, beta1, beta2, eps, loss_kind, delta, loss, grads,
                           ws, (hipStream_t)stream);
}

int cae_mlp_loss_grad(const float *y, const float *target, float *dy, float *loss, uint32_t n, int kind, float delta,
                      void *stream)
{
    if (!y || !target || !dy || !loss) return mfail(CAE_EINVAL, "NULL pointer");
    if (n == 0) return mfail(CAE_EINVAL, "n must be >= 1");
    if (kind != CAE_LOSS_MSE && kind != CAE_LOSS_HUBER) return mfail(CAE_EINVAL, "unknown loss kind");
    if (kind == CAE_LOSS_HUBER && !(delta > 0.0f)) return mfail(CAE_EINVAL, "Huber delta must be > 0");
    hipLaunchKernelGGL(loss_grad, dim3(1), dim3(1024), 0, (hipStream_t)stream, y, target, dy, loss, n, kind, delta);
    return launch_status();
}

}  // extern "C"

namespace {

// The unfused forward pass: x -> bf16, then three matrix-core layer products, activations kept in
// ws (the prefix of ws_layout) for cae_mlp_backward.
int forward_impl(const cae_mlp *net, const float *x, float *y, uint32_t N, void *ws, hipStream_t s)
{
    const uint32_t din = net->d_in, H = net->d_hidden, dout = net->d_out;
    const Layout l = layout(din, H, dout);
    const WsLayout w = ws_layout(din, H, dout, N);
    unsigned char *b = static_cast<unsigned char *>(ws);
    uint16_t *xb = reinterpret_cast<uint16_t *>(b + w.xb);
    float *z1 = reinterpret_cast<float *>(b + w.z1);
    uint16_t *h1 = reinterpret_cast<uint16_t *>(b + w.h1);
    float *z2 = reinterpret_cast<float *>(b + w.z2);
    uint16_t *h2 = reinterpret_cast<uint16_t *>(b + w.h2);
    const uint16_t *W1 = net->weights, *W2 = W1 + (size_t)din * H, *W3 = W2 + (size_t)H * H;
    const uint64_t nx = (uint64_t)N * din;
    hipLaunchKernelGGL(to_bf16, dim3((uint32_t)std::min<uint64_t>((nx + 255) / 256, 1024)), dim3(256), 0, s, x, xb, nx);
    GemmArgs g = gargs(xb, din, W1, H, N, H, din);
    g.bias = net->params + l.b1;
    g.Of = z1;
    g.Ob = h1;
    g.ldo = H;
    gemm<false, false, EPI_HIDDEN>(g, s);
    g = gargs(h1, H, W2, H, N, H, H);
    g.bias = net->params + l.b2;
    g.Of = z2;
    g.Ob = h2;
    g.ldo = H;
    gemm<false, false, EPI_HIDDEN>(g, s);
    g = gargs(h2, H, W3, dout, N, dout, H);
    g.bias = net->params + l.b3;
    g.Of = y;
    g.ldo = dout;
    gemm<false, false, EPI_OUTPUT>(g, s);
    return launch_status();
}

}  // namespace

