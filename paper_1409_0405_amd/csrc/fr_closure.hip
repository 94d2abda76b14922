// Learned closure kernels: per-element P1 moments, network inputs, and a
// small fully connected network (120 -> 64 -> 64 -> 20, tanh) with its
// forward pass, hand-derived backward pass and Adam update.
//
// The closure adds to an order-1 residual the P1 part of the difference
// between the filtered high-order residual and the order-1 residual of the
// filtered state, as predicted from the element's and its face neighbours'
// P1 moments.  Parameter layout: W1 [64][120], b1 [64], W2 [64][64], b2 [64],
// W3 [20][64], b3 [20] (row-major, in this order).
#include <hip/hip_runtime.h>

#include <cmath>

#include "fr_device.hpp"

namespace frd {

namespace {

constexpr int OW1 = 0, OB1 = OW1 + MLP_H * MLP_IN, OW2 = OB1 + MLP_H, OB2 = OW2 + MLP_H * MLP_H;
constexpr int OW3 = OB2 + MLP_H, OB3 = OW3 + MLP_OUT * MLP_H;
static_assert(OB3 + MLP_OUT == MLP_NPARAM, "parameter layout");

// Weight read: FP32 master copy, or its BF16 rounding (stored as the high
// half of the FP32 bit pattern).
template <bool BF16W>
__device__ __forceinline__ float wt(const float *p, const uint16_t *pb, int i) {
    if constexpr (BF16W)
        return __builtin_bit_cast(float, uint32_t(pb[i]) << 16);
    else
        return p[i];
}

// moments mom[g * rs + (v * 4 + a) * cs] = sum_i Mom[a][i] U[i][v][e], g = goff + e
// (element-major rs = 20, cs = 1, or feature-major rs = 1, cs = n_total); of
// U - B when B is given; targets then normalised (m - mu_y) / s_y if ystats
template <typename T>
__global__ __launch_bounds__(256) void moments_kernel(const T *__restrict__ U, const T *__restrict__ B,
                                                      int64_t ld, int64_t nelem, int nu,
                                                      const float *__restrict__ Mom,
                                                      float *__restrict__ mom, int64_t goff, int64_t rs,
                                                      int64_t cs, const float *__restrict__ ystats) {
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= nelem) return;
    float m[20];
#pragma unroll
    for (int q = 0; q < 20; ++q) m[q] = 0;
    for (int i = 0; i < nu; ++i)
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            const int64_t o = (int64_t(i) * 5 + v) * ld + e;
            const float u = B ? float(U[o] - B[o]) : float(U[o]);
#pragma unroll
            for (int a = 0; a < 4; ++a) m[v * 4 + a] += Mom[a * nu + i] * u;
        }
    float *out = mom + (goff + e) * rs;
#pragma unroll
    for (int q = 0; q < 20; ++q) out[q * cs] = ystats ? (m[q] - ystats[q]) / ystats[MLP_OUT + q] : m[q];
}

// inputs x[g][0..119]: own moments, then the neighbours' across faces 0..4
// (zeros where there is no such face), normalised (x - mu) / s if stats.
// Moments at mom[g * rs + q * cs], inputs at feat[g * frs + k * fcs].
__global__ __launch_bounds__(256) void features_kernel(const float *__restrict__ mom, int64_t rs, int64_t cs,
                                                       const int32_t *__restrict__ nb,
                                                       int64_t ntot,
                                                       const float *__restrict__ stats,
                                                       float *__restrict__ feat, int64_t frs, int64_t fcs) {
    const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= ntot) return;
    float *out = feat + g * frs;
    for (int b = 0; b < 6; ++b) {
        const int64_t src = b == 0 ? g : nb[g * 5 + b - 1];
        for (int q = 0; q < 20; ++q) {
            float v = src >= 0 ? mom[src * rs + q * cs] : 0.0f;
            if (stats) v = (v - stats[b * 20 + q]) / stats[MLP_IN + b * 20 + q];
            out[(b * 20 + q) * fcs] = v;
        }
    }
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

// tanh x = 1 - 2 / (1 + e^(2x)) with the hardware base-2 exponential and
// reciprocal: absolute error below 1e-6 over the whole line (e^(2x)
// overflowing to infinity gives 1, underflowing to 0 gives -1)
__device__ __forceinline__ float fast_tanh(float x) {
    const float e = __builtin_amdgcn_exp2f(x * 2.8853900817779268f);   // 2 / ln 2
    return 1.0f - 2.0f * __builtin_amdgcn_rcpf(1.0f + e);
}

// x unchanged but opaque to the optimiser, so that a value loaded ahead of
// a loop stays a separate register set (see the operator-product kernels)
__device__ __forceinline__ float opaque(float x) {
    asm volatile("" : "+v"(x));
    return x;
}

// The network's forward pass on the FP32 matrix cores: one wavefront per 32
// samples, eight per workgroup (two per SIMD).  The workgroup stages the weights (FP32, or
// their BF16 rounding widened to FP32) in LDS.  Each layer is a product of
// 16 x 16 x 4 steps with the samples as rows (A: inputs or activations, lane
// l holding sample l % 16 of a 16-row block at K index l / 16) and the
// transposed weights as B; all output blocks of a layer are accumulated
// together (16 independent accumulators), then bias and tanh are applied on
// the accumulators and the activations go to the wavefront's LDS rows as the
// next layer's A operand.  Inputs at X[s * xrs + k * xcs], outputs at
// Y[s * yrs + o * ycs] (sample-major or feature-major).
constexpr int FWD_HP = MLP_H + 1;                 // padded activation row (no bank conflicts)
constexpr int FWD_WAVES = 8, FWD_MS = 2;          // 8 wavefronts of 32 samples per workgroup
constexpr int FWD_TILE = FWD_WAVES * FWD_MS * 16;
template <bool BF16W>
__global__ __launch_bounds__(512) void mlp_forward_mfma_kernel(const float *__restrict__ P,
                                                               const uint16_t *__restrict__ Pb,
                                                               const float *__restrict__ X, int64_t xrs,
                                                               int64_t xcs, int64_t n,
                                                               const float *__restrict__ stats, bool norm_in,
                                                               float *__restrict__ Y, int64_t yrs, int64_t ycs) {
    // weights in matrix-operand order: layer l, block jb, K step kb, lane ->
    // W_l[16 jb + lane % 16][4 kb + lane / 16] (one conflict-free 256-byte
    // LDS read per operand); layer 3 padded to 32 rows with zeros; biases after
    constexpr int F1 = 0, F2 = F1 + MLP_H * MLP_IN, F3 = F2 + MLP_H * MLP_H, FB = F3 + 32 * MLP_H;
    __shared__ float W[FB + 2 * MLP_H + MLP_OUT];
    __shared__ float Hs[FWD_WAVES][FWD_MS * 16][FWD_HP];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int i = tid; i < FB; i += FWD_WAVES * 64) {
        int base, K, rows, ow;
        if (i < F2) { base = F1; K = MLP_IN; rows = MLP_H; ow = OW1; }
        else if (i < F3) { base = F2; K = MLP_H; rows = MLP_H; ow = OW2; }
        else { base = F3; K = MLP_H; rows = MLP_OUT; ow = OW3; }
        const int q = i - base, l = q & 63, kb = (q >> 6) % (K / 4), jb = (q >> 6) / (K / 4);
        const int row = 16 * jb + (l & 15), col = 4 * kb + (l >> 4);
        W[i] = row < rows ? wt<BF16W>(P, Pb, ow + row * K + col) : 0.0f;
    }
    for (int i = tid; i < 2 * MLP_H + MLP_OUT; i += FWD_WAVES * 64)
        W[FB + i] = wt<BF16W>(P, Pb, i < MLP_H ? OB1 + i : i < 2 * MLP_H ? OB2 + i - MLP_H : OB3 + i - 2 * MLP_H);
    __syncthreads();
    const int r16 = lane & 15, g = lane >> 4;
    // persistent over tiles of 256 samples: the weights are staged once per workgroup
    for (int64_t tile = blockIdx.x; tile * FWD_TILE < n; tile += gridDim.x) {
    const int64_t s0 = (tile * FWD_WAVES + w) * (FWD_MS * 16);
    float(*H)[FWD_HP] = Hs[w];
    f32x4 acc[4][FWD_MS];                          // [output block][sample block]
    auto zero = [&]() {
#pragma unroll
        for (int jb = 0; jb < 4; ++jb)
#pragma unroll
            for (int m = 0; m < FWD_MS; ++m) acc[jb][m] = f32x4{0, 0, 0, 0};
    };
    // layer 1: A straight from the inputs (standardised if asked; samples
    // past n are zero); all 120 values of the lane's operands are loaded
    // up front, so the tile waits for memory once
    zero();
    float xa[MLP_IN / 4][FWD_MS];
#pragma unroll
    for (int kb = 0; kb < MLP_IN / 4; ++kb)
#pragma unroll
        for (int m = 0; m < FWD_MS; ++m) {
            const int64_t sidx = s0 + 16 * m + r16;
            xa[kb][m] = sidx < n ? X[sidx * xrs + int64_t(4 * kb + g) * xcs] : 0.0f;
        }
#pragma unroll
    for (int kb = 0; kb < MLP_IN / 4; ++kb) {
        const int k = 4 * kb + g;
        float a[FWD_MS], b[4];
#pragma unroll
        for (int m = 0; m < FWD_MS; ++m) {
            a[m] = xa[kb][m];
            if (norm_in) a[m] = s0 + 16 * m + r16 < n ? (a[m] - stats[k]) / stats[MLP_IN + k] : 0.0f;
        }
#pragma unroll
        for (int jb = 0; jb < 4; ++jb) b[jb] = W[F1 + (jb * (MLP_IN / 4) + kb) * 64 + lane];
#pragma unroll
        for (int jb = 0; jb < 4; ++jb)
#pragma unroll
            for (int m = 0; m < FWD_MS; ++m) acc[jb][m] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[m], b[jb], acc[jb][m], 0, 0, 0);
    }
    auto to_h = [&](int ob) {
#pragma unroll
        for (int jb = 0; jb < 4; ++jb) {
            const int j = 16 * jb + r16;
            const float bias = W[FB + ob + j];
#pragma unroll
            for (int m = 0; m < FWD_MS; ++m)
#pragma unroll
                for (int r = 0; r < 4; ++r) H[16 * m + 4 * g + r][j] = fast_tanh(acc[jb][m][r] + bias);
        }
    };
    to_h(0);
    __syncthreads();
    // layer 2: A from the activations; the results stay in the accumulators
    // until every lane of the wavefront has read its operands, then replace them
    zero();
    for (int kb = 0; kb < MLP_H / 4; ++kb) {
        const int k = 4 * kb + g;
        float a[FWD_MS], b[4];
#pragma unroll
        for (int m = 0; m < FWD_MS; ++m) a[m] = H[16 * m + r16][k];
#pragma unroll
        for (int jb = 0; jb < 4; ++jb) b[jb] = W[F2 + (jb * (MLP_H / 4) + kb) * 64 + lane];
#pragma unroll
        for (int jb = 0; jb < 4; ++jb)
#pragma unroll
            for (int m = 0; m < FWD_MS; ++m) acc[jb][m] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[m], b[jb], acc[jb][m], 0, 0, 0);
    }
    __syncthreads();
    to_h(MLP_H);
    __syncthreads();
    // layer 3: 20 outputs in two blocks of 16 (the last 12 columns are zero
    // weights and are not stored)
    zero();
    for (int kb = 0; kb < MLP_H / 4; ++kb) {
        const int k = 4 * kb + g;
        float a[FWD_MS], b[2];
#pragma unroll
        for (int m = 0; m < FWD_MS; ++m) a[m] = H[16 * m + r16][k];
#pragma unroll
        for (int jb = 0; jb < 2; ++jb) b[jb] = W[F3 + (jb * (MLP_H / 4) + kb) * 64 + lane];
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
            for (int m = 0; m < FWD_MS; ++m) acc[jb][m] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[m], b[jb], acc[jb][m], 0, 0, 0);
    }
#pragma unroll
    for (int jb = 0; jb < 2; ++jb) {
        const int o = 16 * jb + r16;
        if (o >= MLP_OUT) continue;
        const float bias = W[FB + 2 * MLP_H + o];
        const float sc = stats ? stats[2 * MLP_IN + MLP_OUT + o] : 1.0f;
        const float mu = stats ? stats[2 * MLP_IN + o] : 0.0f;
#pragma unroll
        for (int m = 0; m < FWD_MS; ++m)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t sidx = s0 + 16 * m + 4 * g + r;
                if (sidx < n) {
                    float z = acc[jb][m][r] + bias;
                    if (stats) z = z * sc + mu;
                    Y[sidx * yrs + int64_t(o) * ycs] = z;
                }
            }
    }
    __syncthreads();           // H is rewritten by the next tile
    }
}

// Gradient of L = sum_s |y_s - t_s|^2 / n over the samples idx[0..n) (or
// 0..n), FP32 master weights; with stats, rows are standardised on load
// (x - mu_x) / s_x and (t - mu_y) / s_y.  Each block (one wavefront) takes chunks of 64
// samples: every lane runs one sample forward and backward, stages the
// per-sample vectors in shared memory, then every lane sums the outer
// products of the parameters it owns over the chunk into the block's
// partial-gradient row (entry MLP_NPARAM holds the partial loss).
__global__ __launch_bounds__(64) void mlp_grad_kernel(const float *__restrict__ P,
                                                      const float *__restrict__ X,
                                                      const float *__restrict__ Tg,
                                                      const int32_t *__restrict__ idx,
                                                      int64_t n, const float *__restrict__ stats,
                                                      float *__restrict__ partial) {
    __shared__ float Xs[64][MLP_IN];
    __shared__ float H1[64][MLP_H], H2[64][MLP_H], D1[64][MLP_H], D2[64][MLP_H], DY[64][MLP_OUT];
    const int tid = threadIdx.x;
    float *part = partial + int64_t(blockIdx.x) * (MLP_NPARAM + 1);
    for (int p = tid; p <= MLP_NPARAM; p += 64) part[p] = 0.0f;
    __syncthreads();
    const float inv_n = 1.0f / float(n);
    for (int64_t c0 = int64_t(blockIdx.x) * 64; c0 < n; c0 += int64_t(gridDim.x) * 64) {
        const int64_t s = c0 + tid;
        const bool live = s < n;
        const int64_t row = live ? (idx ? int64_t(idx[s]) : s) : 0;
        for (int k = 0; k < MLP_IN; ++k) {
            float x = live ? X[row * MLP_IN + k] : 0.0f;
            if (stats && live) x = (x - stats[k]) / stats[MLP_IN + k];
            Xs[tid][k] = x;
        }
        for (int j = 0; j < MLP_H; ++j) {
            float z = P[OB1 + j];
            for (int k = 0; k < MLP_IN; ++k) z += P[OW1 + j * MLP_IN + k] * Xs[tid][k];
            H1[tid][j] = tanhf(z);
        }
        for (int j = 0; j < MLP_H; ++j) {
            float z = P[OB2 + j];
            for (int k = 0; k < MLP_H; ++k) z += P[OW2 + j * MLP_H + k] * H1[tid][k];
            H2[tid][j] = tanhf(z);
        }
        float loss = 0.0f;
        for (int o = 0; o < MLP_OUT; ++o) {
            float z = P[OB3 + o];
            for (int k = 0; k < MLP_H; ++k) z += P[OW3 + o * MLP_H + k] * H2[tid][k];
            float t = live ? Tg[row * MLP_OUT + o] : 0.0f;
            if (stats) t = (t - stats[2 * MLP_IN + o]) / stats[2 * MLP_IN + MLP_OUT + o];
            const float d = live ? z - t : 0.0f;
            loss += d * d;
            DY[tid][o] = 2.0f * d * inv_n;
        }
        for (int j = 0; j < MLP_H; ++j) {          // dz2 = (W3^T dy) (1 - h2^2)
            float a = 0.0f;
            for (int o = 0; o < MLP_OUT; ++o) a += P[OW3 + o * MLP_H + j] * DY[tid][o];
            D2[tid][j] = a * (1.0f - H2[tid][j] * H2[tid][j]);
        }
        for (int j = 0; j < MLP_H; ++j) {          // dz1 = (W2^T dz2) (1 - h1^2)
            float a = 0.0f;
            for (int k = 0; k < MLP_H; ++k) a += P[OW2 + k * MLP_H + j] * D2[tid][k];
            D1[tid][j] = a * (1.0f - H1[tid][j] * H1[tid][j]);
        }
        __syncthreads();
        // outer products summed over the chunk; lane tid owns every 64th parameter
        for (int p = tid; p < MLP_NPARAM; p += 64) {
            float a = 0.0f;
            if (p < OB1) {
                const int j = p / MLP_IN, k = p % MLP_IN;
                for (int q = 0; q < 64; ++q) a += D1[q][j] * Xs[q][k];
            } else if (p < OW2) {
                for (int q = 0; q < 64; ++q) a += D1[q][p - OB1];
            } else if (p < OB2) {
                const int j = (p - OW2) / MLP_H, k = (p - OW2) % MLP_H;
                for (int q = 0; q < 64; ++q) a += D2[q][j] * H1[q][k];
            } else if (p < OW3) {
                for (int q = 0; q < 64; ++q) a += D2[q][p - OB2];
            } else if (p < OB3) {
                const int o = (p - OW3) / MLP_H, k = (p - OW3) % MLP_H;
                for (int q = 0; q < 64; ++q) a += DY[q][o] * H2[q][k];
            } else {
                for (int q = 0; q < 64; ++q) a += DY[q][p - OB3];
            }
            part[p] += a;
        }
        // partial loss: lane 0 sums the chunk's per-lane losses through shared memory
        __syncthreads();
        H1[tid][0] = loss;
        __syncthreads();
        if (tid == 0) {
            float l = 0.0f;
            for (int q = 0; q < 64; ++q) l += H1[q][0];
            part[MLP_NPARAM] += l * inv_n;
        }
        __syncthreads();
    }
}

// grad[p] = sum over blocks of partial[b][p], blocks in order
__global__ __launch_bounds__(256) void mlp_reduce_kernel(const float *__restrict__ partial,
                                                         int nblk, float *__restrict__ grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > MLP_NPARAM) return;
    float s = 0.0f;
    for (int b = 0; b < nblk; ++b) s += partial[int64_t(b) * (MLP_NPARAM + 1) + p];
    grad[p] = s;
}

// Adam (Kingma & Ba): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
// p -= lr (m / c1) / (sqrt(v / c2) + eps); also refresh the BF16 copy.
__global__ __launch_bounds__(256) void adam_kernel(float *__restrict__ P, const float *__restrict__ G,
                                                   float *__restrict__ M, float *__restrict__ V,
                                                   float lr, float b1, float b2, float eps, float c1,
                                                   float c2, uint16_t *__restrict__ Pb) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= MLP_NPARAM) return;
    const float g = G[p];
    const float m = b1 * M[p] + (1.0f - b1) * g;
    const float v = b2 * V[p] + (1.0f - b2) * g * g;
    M[p] = m;
    V[p] = v;
    const float w = P[p] - lr * (m / c1) / (sqrtf(v / c2) + eps);
    P[p] = w;
    uint32_t b = __builtin_bit_cast(uint32_t, w);
    b += 0x7fffu + ((b >> 16) & 1u);   // round to nearest even
    Pb[p] = uint16_t(b >> 16);
}

__global__ __launch_bounds__(256) void to_bf16_kernel(const float *__restrict__ P, uint16_t *__restrict__ Pb) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= MLP_NPARAM) return;
    uint32_t b = __builtin_bit_cast(uint32_t, P[p]);
    b += 0x7fffu + ((b >> 16) & 1u);
    Pb[p] = uint16_t(b >> 16);
}

}  // namespace

template <typename T>
hipError_t launch_moments(const T *U, const T *B, int64_t ld, int64_t nelem, int nu, const float *Mom,
                          float *mom, int64_t goff, int64_t rs, int64_t cs, const float *ystats,
                          hipStream_t s) {
    if (!nelem) return hipSuccess;
    moments_kernel<T><<<unsigned((nelem + 255) / 256), 256, 0, s>>>(U, B, ld, nelem, nu, Mom, mom, goff, rs,
                                                                    cs, ystats);
    return hipGetLastError();
}

hipError_t launch_features(const float *mom, int64_t rs, int64_t cs, const int32_t *nb, int64_t ntot,
                           const float *stats, float *feat, int64_t frs, int64_t fcs, hipStream_t s) {
    if (!ntot) return hipSuccess;
    features_kernel<<<unsigned((ntot + 255) / 256), 256, 0, s>>>(mom, rs, cs, nb, ntot, stats, feat, frs, fcs);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const float *P, const uint16_t *Pb, bool bf16, const float *X, int64_t xrs,
                              int64_t xcs, int64_t n, const float *stats, bool norm_in, float *Y, int64_t yrs,
                              int64_t ycs, hipStream_t s) {
    if (!n) return hipSuccess;
    // one workgroup per CU (the staged weights and activations take 119 KB
    // of LDS), each looping over tiles of FWD_TILE samples
    const int64_t tiles = (n + FWD_TILE - 1) / FWD_TILE;
    const unsigned g = unsigned(tiles < 256 ? tiles : 256);
    norm_in = norm_in && stats;
    if (bf16)
        mlp_forward_mfma_kernel<true><<<g, FWD_WAVES * 64, 0, s>>>(P, Pb, X, xrs, xcs, n, stats, norm_in, Y, yrs, ycs);
    else
        mlp_forward_mfma_kernel<false><<<g, FWD_WAVES * 64, 0, s>>>(P, Pb, X, xrs, xcs, n, stats, norm_in, Y, yrs,
                                                                   ycs);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const float *P, const float *X, const float *Tg, const int32_t *idx, int64_t n,
                           const float *stats, float *partial, int nblk, float *grad, hipStream_t s) {
    if (n <= 0) return hipErrorInvalidValue;
    const int64_t chunks = (n + 63) / 64;
    const int g = int(chunks < nblk ? chunks : nblk);
    mlp_grad_kernel<<<g, 64, 0, s>>>(P, X, Tg, idx, n, stats, partial);
    mlp_reduce_kernel<<<(MLP_NPARAM + 256) / 256, 256, 0, s>>>(partial, g, grad);
    return hipGetLastError();
}

hipError_t launch_adam(float *P, const float *G, float *M, float *V, float lr, float b1, float b2, float eps,
                       int t, uint16_t *Pb, hipStream_t s) {
    const float c1 = 1.0f - powf(b1, float(t)), c2 = 1.0f - powf(b2, float(t));
    adam_kernel<<<(MLP_NPARAM + 255) / 256, 256, 0, s>>>(P, G, M, V, lr, b1, b2, eps, c1, c2, Pb);
    return hipGetLastError();
}

hipError_t launch_to_bf16(const float *P, uint16_t *Pb, hipStream_t s) {
    to_bf16_kernel<<<(MLP_NPARAM + 255) / 256, 256, 0, s>>>(P, Pb);
    return hipGetLastError();
}

template hipError_t launch_moments<float>(const float *, const float *, int64_t, int64_t, int, const float *,
                                          float *, int64_t, int64_t, int64_t, const float *, hipStream_t);
template hipError_t launch_moments<double>(const double *, const double *, int64_t, int64_t, int,
                                           const float *, float *, int64_t, int64_t, int64_t, const float *,
                                           hipStream_t);

}  // namespace frd
