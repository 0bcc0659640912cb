// axpic_mlp.hip -- the rate surrogate on gfx950 matrix cores.
//
// A perceptron 8 -> 128 -> 128 -> 128 -> 128 -> 1 with hard-swish
// activations predicts the residual y of the logarithm of a rate,
// log R = mu_ch + lin_ch . f + sigma_ch * y, from the normalised features f of
// (log(omega/T), log(kappa/T), log n_e, Z) and a channel one-hot.  Weights and
// layer inputs are bfloat16, accumulation FP32 (v_mfma_f32_16x16x32_bf16).
// Hard-swish costs two vector instructions (an FMA with clamp, a multiply):
// the inference stays bound by the matrix cores, where a sigmoid-based
// activation (an exponential and a reciprocal per element) would leave it
// bound by the vector ALU.
//
// Training (forward with saved activations, backward, Adam on FP32 master
// weights) uses one generic MFMA GEMM kernel plus elementwise kernels.  The
// inference kernel keeps the whole network in LDS in MFMA-fragment order and
// chains the layers in registers: it computes H^T = W^T X^T with the
// particles as the MFMA column dimension, so each layer's accumulator
// registers are, after activation and rounding, the next layer's B operand
// under a fixed permutation of the feature index that the packed weights
// follow.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>

#include "../../include/axpic.h"
#include "axpic_device.hpp"
#include "axpic_timing.hpp"

using namespace axpic;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

namespace {

// padded widths of the training layout
constexpr int kD0 = 32, kDH = 128, kD5 = 32;
constexpr int kSplitMax = 16;              // K splits of a training GEMM at most
// offsets of the FP32 master parameters
constexpr int64_t kOffW1 = 0;
constexpr int64_t kOffB1 = kOffW1 + kD0 * kDH;
constexpr int64_t kOffW2 = kOffB1 + kDH;
constexpr int64_t kLayerHH = kDH * kDH + kDH;        // W + b of a hidden 128x128 layer
constexpr int64_t kOffW5 = kOffW2 + 3 * kLayerHH;
constexpr int64_t kOffB5 = kOffW5 + kDH * kD5;
constexpr int64_t kNParams = kOffB5 + kD5;
static_assert(kNParams == AXPIC_MLP_PARAMS, "parameter layout");

inline int64_t offW(int l) { return l == 1 ? kOffW1 : (l == 5 ? kOffW5 : kOffW2 + (l - 2) * kLayerHH); }
inline int64_t offB(int l) { return l == 1 ? kOffB1 : (l == 5 ? kOffB5 : kOffW2 + (l - 2) * kLayerHH + kDH * kDH); }
inline int dIn(int l) { return l == 1 ? kD0 : kDH; }
inline int dOut(int l) { return l == 5 ? kD5 : kDH; }

// inference blob: 108 fragments of 64 lanes x 8 bf16, then FP32 biases
constexpr int kFragL1 = 0, kFragL2 = 8, kFragL5 = 8 + 96, kNFrag = 8 + 96 + 4;
constexpr int kFragBytes = 64 * 8 * 2;
constexpr int kBiasFloats = 4 * kDH + 16;
constexpr size_t kBlobBytes = (size_t)kNFrag * kFragBytes + sizeof(float) * kBiasFloats;
static_assert(kBlobBytes == AXPIC_MLP_BLOB_BYTES, "blob layout");

inline hipStream_t S(void* s) { return (hipStream_t)s; }
inline axpic_status launched() { return hipGetLastError() == hipSuccess ? AXPIC_OK : AXPIC_E_DEVICE; }

// hard-swish h(z) = z clamp(z/6 + 1/2, 0, 1) and its derivative
__device__ __forceinline__ float act(float z) {
    return z * __builtin_amdgcn_fmed3f(fmaf(z, 1.0f / 6.0f, 0.5f), 0.0f, 1.0f);
}
__device__ __forceinline__ float dact(float z) {
    const float t = __builtin_amdgcn_fmed3f(fmaf(z, 1.0f / 6.0f, 0.5f), 0.0f, 1.0f);
    return (z > -3.0f && z < 3.0f) ? fmaf(z, 1.0f / 6.0f, t) : t;
}

// ------------------------------------------------------------------ training GEMM
// C[M x N] = op(A)[M x K] op(B)[K x N] (+ bias[N]); A(m,k) = transA ? A[k lda + m] : A[m lda + k],
// B(k,n) = transB ? B[n ldb + k] : B[k ldb + n].  Operands rounded to bf16, FP32 accumulation.
// A workgroup of four wavefronts computes a 32 x 32 tile of C, each wavefront a 16 x 16
// quarter: per 32-deep slice of K, op(A) and op(B) are read once from global memory in
// 16-byte loads along their contiguous dimension, rounded to bf16 and stored k-contiguous
// in LDS (rows padded against bank conflicts), from where each wavefront takes its MFMA
// operands.  With gridDim.z > 1 the K range is split: slice z adds up K / gridDim.z and
// writes its partial tile to C + z M N (no bias), summed in order by k_gemm_splitk_sum.
// M, N multiples of 32, K a multiple of 32 gridDim.z; lda, ldb multiples of 4.
constexpr int kGemmPad = 40;               // bf16 per LDS row: 32 + 8
__device__ __forceinline__ void gemm_stage(const float* __restrict__ X, int64_t ld, int trans,
                                           int64_t r0, int64_t k0, __bf16 (*S)[kGemmPad]) {
    // 32 x 32 slice X(r0 .., k0 ..) of op(X) (op(X)(r, k) = trans ? X[k ld + r] : X[r ld + k])
    // into S[r][k]: thread t loads four consecutive floats along X's contiguous dimension
    const int t = threadIdx.x, u = t >> 3, v = (t & 7) * 4;
    if (!trans) {
        const float4 q = *(const float4*)(X + (r0 + u) * ld + k0 + v);
        S[u][v] = (__bf16)q.x; S[u][v + 1] = (__bf16)q.y; S[u][v + 2] = (__bf16)q.z; S[u][v + 3] = (__bf16)q.w;
    } else {
        const float4 q = *(const float4*)(X + (k0 + u) * ld + r0 + v);
        S[v][u] = (__bf16)q.x; S[v + 1][u] = (__bf16)q.y; S[v + 2][u] = (__bf16)q.z; S[v + 3][u] = (__bf16)q.w;
    }
}

__global__ void __launch_bounds__(256)
k_gemm_bf16(int64_t M, int64_t N, int64_t K, const float* __restrict__ A, int64_t lda, int transA,
            const float* __restrict__ B, int64_t ldb, int transB, float* __restrict__ C,
            int64_t ldc, const float* __restrict__ bias) {
    __shared__ __bf16 As[32][kGemmPad], Bs[32][kGemmPad];
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6, g = l >> 4;
    const int64_t m0 = (int64_t)blockIdx.y * 32, n0 = (int64_t)blockIdx.x * 32;
    const int wm = (w >> 1) * 16, wn = (w & 1) * 16;
    const int64_t kz = K / gridDim.z, kb = kz * blockIdx.z;
    floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int64_t k0 = kb; k0 < kb + kz; k0 += 32) {
        gemm_stage(A, lda, transA, m0, k0, As);
        gemm_stage(B, ldb, !transB, n0, k0, Bs);     // Bs[n][k] = op(B)(k, n)
        __syncthreads();
        bf16x8 a, b;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            a[j] = As[wm + (l & 15)][8 * g + j];
            b[j] = Bs[wn + (l & 15)][8 * g + j];
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
        __syncthreads();
    }
    const int64_t n = n0 + wn + (l & 15);
    if (gridDim.z == 1) {
        const float bv = bias ? bias[n] : 0.0f;
#pragma unroll
        for (int r = 0; r < 4; ++r) C[(m0 + wm + 4 * g + r) * ldc + n] = acc[r] + bv;
    } else {
        float* P = C + (int64_t)blockIdx.z * M * N;
#pragma unroll
        for (int r = 0; r < 4; ++r) P[(m0 + wm + 4 * g + r) * N + n] = acc[r];
    }
}

// C[m][n] = sum over the split partials in order (+ bias[n]).
__global__ void __launch_bounds__(256)
k_gemm_splitk_sum(int64_t M, int64_t N, int nsplit, const float* __restrict__ P,
                  float* __restrict__ C, int64_t ldc, const float* __restrict__ bias) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M * N) return;
    const int64_t m = i / N, n = i - m * N;
    float s = 0.0f;
    for (int z = 0; z < nsplit; ++z) s += P[(int64_t)z * M * N + i];
    C[m * ldc + n] = s + (bias ? bias[n] : 0.0f);
}

// The same product in FP32 throughout (the training calls' FP32-weight mode, for
// gradient checks at FP32 accuracy): 16 x 16 output tiles per workgroup of 256
// threads, 16-deep slices of op(A) and op(B) staged in LDS, one fused multiply-add
// per k in increasing k order.
__global__ void __launch_bounds__(256)
k_gemm_f32(int64_t M, int64_t N, int64_t K, const float* __restrict__ A, int64_t lda, int transA,
           const float* __restrict__ B, int64_t ldb, int transB, float* __restrict__ C,
           int64_t ldc, const float* __restrict__ bias) {
    __shared__ float As[16][17], Bs[16][17];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int64_t m = (int64_t)blockIdx.y * 16 + ty, n = (int64_t)blockIdx.x * 16 + tx;
    float acc = 0.0f;
    for (int64_t k0 = 0; k0 < K; k0 += 16) {
        // As[ty][tx] = op(A)(m, k0 + tx), Bs[ty][tx] = op(B)(k0 + ty, n)
        const int64_t ka = k0 + tx, kb = k0 + ty;
        As[ty][tx] = transA ? A[ka * lda + m] : A[m * lda + ka];
        Bs[ty][tx] = transB ? B[n * ldb + kb] : B[kb * ldb + n];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 16; ++k) acc = fmaf(As[ty][k], Bs[k][tx], acc);
        __syncthreads();
    }
    C[m * ldc + n] = acc + (bias ? bias[n] : 0.0f);
}

__global__ void __launch_bounds__(256)
k_act_fwd(int64_t n, const float* __restrict__ Z, float* __restrict__ H) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) H[i] = act(Z[i]);
}

__global__ void __launch_bounds__(256)
k_act_bwd(int64_t n, const float* __restrict__ Z, float* __restrict__ dZ) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dZ[i] = dZ[i] * dact(Z[i]);
}

// dZ5 = 2 (y - Y)/B in column 0 (the padded columns carry no gradient); loss partials.
__global__ void __launch_bounds__(256)
k_mse_grad(int64_t Bn, const float* __restrict__ Z5, const float* __restrict__ Y,
           float* __restrict__ dZ5, double* __restrict__ loss) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double e2 = 0.0;
    if (b < Bn) {
        // a row with a NaN target (no valid label) carries no gradient and no loss
        const float r = isnan(Y[b]) ? 0.0f : Z5[b * kD5] - Y[b];
        for (int c = 0; c < kD5; ++c) dZ5[b * kD5 + c] = c == 0 ? 2.0f * r / (float)Bn : 0.0f;
        e2 = (double)r * r;
    }
    e2 = wave_sum(e2);
    if ((threadIdx.x & 63) == 0 && loss) atomicAdd(loss, e2 / (double)Bn);
}

// Column sums (bias gradients): one workgroup per column, fixed reduction order.
__global__ void __launch_bounds__(256)
k_colsum(int64_t Bn, int64_t N, const float* __restrict__ dZ, float* __restrict__ out) {
    __shared__ float part[4];
    const int64_t c = blockIdx.x;
    float s = 0.0f;
    for (int64_t b = threadIdx.x; b < Bn; b += 256) s += dZ[b * N + c];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[c] = part[0] + part[1] + part[2] + part[3];
}

__global__ void k_zero_d(double* p) { if (threadIdx.x == 0) *p = 0.0; }

__global__ void __launch_bounds__(256)
k_col0(int64_t Bn, const float* __restrict__ Z5, float* __restrict__ y) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b < Bn) y[b] = Z5[b * kD5];
}

__global__ void __launch_bounds__(256)
k_adam(int64_t n, float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi; v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ------------------------------------------------------------------ training set
// Rows with a non-finite label (brems samples whose screening factor is not
// positive) take part in no statistic and carry a NaN target, which the loss skips.
constexpr int kPrepBlocks = 256;
constexpr int kMomN = 21;   // per channel: 15 of d d^T (upper triangle), 5 of d y, y y; d = (1, f)

// Per-block minimum and maximum of the raw features 0..2 over the valid rows.
__global__ void __launch_bounds__(256)
k_prep_range(int64_t n, const double* __restrict__ feat, const double* __restrict__ logR,
             double* __restrict__ part) {
    __shared__ double red[256];
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        if (!isfinite(logR[i])) continue;
        for (int k = 0; k < 3; ++k) { mn[k] = fmin(mn[k], feat[4 * i + k]); mx[k] = fmax(mx[k], feat[4 * i + k]); }
    }
    for (int q = 0; q < 6; ++q) {
        red[threadIdx.x] = q < 3 ? mn[q] : mx[q - 3];
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o)
                red[threadIdx.x] = q < 3 ? fmin(red[threadIdx.x], red[threadIdx.x + o])
                                         : fmax(red[threadIdx.x], red[threadIdx.x + o]);
            __syncthreads();
        }
        if (threadIdx.x == 0) part[blockIdx.x * 6 + q] = red[0];
        __syncthreads();
    }
}

struct PrepNorm { double lo[4], sc[4], mu[4], lin[4][4], sigma[4]; };

__device__ __forceinline__ void prep_features(const double* __restrict__ f, const PrepNorm& nm,
                                              double* fn) {
    for (int k = 0; k < 4; ++k) fn[k] = (f[k] - nm.lo[k]) * nm.sc[k] - 1.0;
}

// Per-block sums of d d^T, d y and y y over the valid rows of channel c, d = (1, f(x)).
__global__ void __launch_bounds__(256)
k_prep_moments(int64_t n, const double* __restrict__ feat, const double* __restrict__ logR,
               const int32_t* __restrict__ ch, int c, PrepNorm nm, double* __restrict__ part) {
    __shared__ double red[256];
    double acc[kMomN];
    for (int q = 0; q < kMomN; ++q) acc[q] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double y = logR[i];
        if (ch[i] != c || !isfinite(y)) continue;
        double d[5];
        d[0] = 1.0;
        prep_features(feat + 4 * i, nm, d + 1);
        int q = 0;
        for (int a = 0; a < 5; ++a)
            for (int b = a; b < 5; ++b) acc[q++] += d[a] * d[b];
        for (int a = 0; a < 5; ++a) acc[15 + a] += d[a] * y;
        acc[20] += y * y;
    }
    for (int q = 0; q < kMomN; ++q) {
        red[threadIdx.x] = acc[q];
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[blockIdx.x * kMomN + q] = red[0];
        __syncthreads();
    }
}

// Column sums of the per-block partials, in block order: out[q] = sum_b part[b][q].
__global__ void k_prep_sum(int nb, int m, const double* __restrict__ part, double* __restrict__ out,
                           int minmax) {
    const int q = threadIdx.x;
    if (q >= m) return;
    double v = part[q];
    for (int b = 1; b < nb; ++b) {
        const double x = part[b * m + q];
        v = minmax == 0 ? v + x : (q < m / 2 ? fmin(v, x) : fmax(v, x));
    }
    out[q] = v;
}

// Training rows: X [n][32] = (f(x), channel one-hot, zeros), Y = (log R - baseline) / sigma
// (NaN for an invalid row).
__global__ void __launch_bounds__(256)
k_prep_design(int64_t n, const double* __restrict__ feat, const double* __restrict__ logR,
              const int32_t* __restrict__ ch, PrepNorm nm, float* __restrict__ X,
              float* __restrict__ Y) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double fn[4];
    prep_features(feat + 4 * i, nm, fn);
    const int c = ch[i];
    float row[32];
    for (int k = 0; k < 32; ++k) row[k] = 0.0f;
    for (int k = 0; k < 4; ++k) row[k] = (float)fn[k];
    if (c >= 0 && c < 4) row[4 + c] = 1.0f;
    for (int k = 0; k < 32; k += 4)
        *(float4*)(X + i * 32 + k) = make_float4(row[k], row[k + 1], row[k + 2], row[k + 3]);
    const double y = logR[i];
    float t = NAN;
    if (isfinite(y) && c >= 0 && c < 4) {
        double base = nm.mu[c];
        for (int k = 0; k < 4; ++k) base += nm.lin[c][k] * (double)row[k];
        t = (float)((y - base) / nm.sigma[c]);
    }
    Y[i] = t;
}

// A minibatch of rows drawn with replacement: row r_b = floor(u32 n / 2^32) with u32 the
// first word of Philox4x32-10 at counter (b, step, 0x4D4C5042, 0) under key seed.
__global__ void __launch_bounds__(256)
k_prep_batch(int64_t n, const float* __restrict__ X, const float* __restrict__ Y, int64_t batch,
             uint32_t seed_lo, uint32_t seed_hi, int64_t step, float* __restrict__ Xb,
             float* __restrict__ Yb) {
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (b >= batch) return;
    const uint4 r = philox4x32_10(make_uint4((uint32_t)b, (uint32_t)(b >> 32), (uint32_t)step,
                                             0x4D4C5042u), seed_lo, seed_hi);
    const int64_t row = (int64_t)(((uint64_t)r.x * (uint64_t)n) >> 32);
    for (int k = 0; k < 32; k += 4) *(float4*)(Xb + b * 32 + k) = *(const float4*)(X + row * 32 + k);
    Yb[b] = Y[row];
}

// ------------------------------------------------------------------ packing
// Fragment (layer, mt, c), lane l (row m = l%16 of output tile mt, group g = l/16),
// slot j holds W[in = perm(c, g, j)][out = 16 mt + m], rounded to bf16, where
// layer 1: perm = 8 g + j; later layers: perm = 32 c + (j < 4 ? 4 g + j : 16 + 4 g + j - 4).
__device__ __forceinline__ int perm_in(int layer, int c, int g, int j) {
    if (layer == 1) return 8 * g + j;
    return 32 * c + (j < 4 ? 4 * g + j : 16 + 4 * g + (j - 4));
}

__global__ void __launch_bounds__(64)
k_mlp_pack(const float* __restrict__ P, __bf16* __restrict__ frag, float* __restrict__ bias) {
    const int f = blockIdx.x, l = threadIdx.x;
    int layer, mt, c;
    if (f < kFragL2) { layer = 1; mt = f; c = 0; }
    else if (f < kFragL5) { const int q = f - kFragL2; layer = 2 + q / 32; mt = (q % 32) / 4; c = q % 4; }
    else { layer = 5; mt = 0; c = f - kFragL5; }
    const int m = l & 15, g = l >> 4;
    const int out = 16 * mt + m;
    const int64_t ow = layer == 1 ? 0 : (layer == 5 ? kOffW5 : kOffW2 + (layer - 2) * kLayerHH);
    const int dout = layer == 5 ? kD5 : kDH;
    for (int j = 0; j < 8; ++j) {
        const int in = perm_in(layer, c, g, j);
        frag[((int64_t)f * 64 + l) * 8 + j] = (__bf16)P[ow + (int64_t)in * dout + out];
    }
    if (f == 0) {
        for (int k = l; k < 4 * kDH; k += 64) {
            const int layer2 = 1 + k / kDH, o = k % kDH;
            const int64_t ob = layer2 == 1 ? kOffB1 : kOffW2 + (layer2 - 2) * kLayerHH + kDH * kDH;
            bias[k] = P[ob + o];
        }
        if (l < 16) bias[4 * kDH + l] = P[kOffB5 + l];
    }
}

// ------------------------------------------------------------------ inference
constexpr int kInfThreads = 512;            // 8 wavefronts share one copy of the weights
constexpr int kInfThreadsP = 512;           // the same, per-particle kernel
constexpr int kNTTable = 4;                // the same for the per-cell table kernel
// Features that differ between the particles (or rows) of a pass: ln(omega/T), the
// screening scale and ln n_e; the ion charge and the channel's one-hot inputs are
// uniform over the launch or the pass.
constexpr int kVarFeat = 3;

struct MlpConst {
    float feat_lo[4], feat_sc[4];
    float out_mu[4], out_sigma[4];
    float out_lin[4][4];
    double T_lo, T_hi, ne_lo, ne_hi, x_lo, x_hi;
};

// Activated output tile mt (rows 16 mt + 4 g + r of this lane) into the next
// layer's B operand: slot r (mt even) or 4 + r (mt odd) of K-chunk mt/2.
template <int NT>
__device__ __forceinline__ void act_tile(const floatx4 (&a)[NT], int mt, bf16x8 (&Bout)[NT][4]) {
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
#pragma unroll
        for (int r = 0; r < 4; ++r) Bout[nt][mt >> 1][(mt & 1) * 4 + r] = (__bf16)act(a[nt][r]);
    }
}

// One hidden layer, software-pipelined over the 8 output tiles: the products of
// tile mt are issued before the activation of tile mt - 1, so a wavefront's
// vector work overlaps its own matrix-core chain; each weight fragment is read
// from LDS one K-chunk ahead of its products (the scheduling barriers keep the
// read before the previous chunk's products, so its latency hides behind them).
template <int NT>
__device__ __forceinline__ void hidden_layer(const bf16x8* __restrict__ frag, int fbase,
                                             const floatx4* __restrict__ b4, int l, int g,
                                             const bf16x8 (&Bin)[NT][4], bf16x8 (&Bout)[NT][4]) {
    floatx4 a0[NT], a1[NT];
    bf16x8 w = frag[fbase * 64 + l];
#pragma unroll
    for (int mt = 0; mt < 8; ++mt) {
        floatx4 (&acc)[NT] = (mt & 1) ? a1 : a0;
        const floatx4 bv = b4[4 * mt + g];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int nxt = mt * 4 + c + 1;
            bf16x8 wn = w;
            if (nxt < 32) wn = frag[(fbase + nxt) * 64 + l];
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, Bin[nt][c],
                                                                  c == 0 ? bv : acc[nt], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
            w = wn;
        }
        if (mt > 0) act_tile((mt & 1) ? a0 : a1, mt - 1, Bout);
    }
    act_tile(a1, 7, Bout);
}

// One network pass over 16 NT particles of a wavefront: lanes base ..
// base + 16 NT - 1 supply the features f[0..7] of their particle; those lanes
// receive y (the other lanes' return value is unspecified).
template <int NT>
__device__ __forceinline__ float mlp_pass(const bf16x8* __restrict__ frag,
                                          const float* __restrict__ bias, const float f[8],
                                          int base) {
    const int l = threadIdx.x & 63, g = l >> 4, col = l & 15;
    // layer-1 B operand: group 0 of column tile nt carries the 8 features of particle
    // base + 16 nt + col; the other groups hold the zero padding of inputs 8..31.  Only
    // the first kVarFeat features differ between particles: the charge and the channel's
    // one-hot inputs are the same in every lane and need no shuffle.
    bf16x8 B0[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const float v = j < kVarFeat ? __shfl(f[j], base + nt * 16 + col, 64) : f[j];
            B0[nt][j] = (__bf16)(g == 0 ? v : 0.0f);
        }
    }
    bf16x8 Ba[NT][4], Bb[NT][4];
    // layer 1 (one K-chunk), pipelined like the hidden layers
    {
        const floatx4* b4 = (const floatx4*)bias;
        floatx4 a0[NT], a1[NT];
        bf16x8 an = frag[kFragL1 * 64 + l];
#pragma unroll
        for (int mt = 0; mt < 8; ++mt) {
            const bf16x8 a = an;                   // read one tile ahead, as in hidden_layer
            if (mt < 7) an = frag[(kFragL1 + mt + 1) * 64 + l];
            const floatx4 bv = b4[4 * mt + g];
            __builtin_amdgcn_sched_barrier(0);
            if (mt & 1) {
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) a1[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, B0[nt], bv, 0, 0, 0);
                act_tile(a0, mt - 1, Ba);
            } else {
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) a0[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, B0[nt], bv, 0, 0, 0);
                if (mt > 0) act_tile(a1, mt - 1, Ba);
            }
        }
        act_tile(a1, 7, Ba);
    }
#pragma unroll 1
    for (int h = 0; h < 3; ++h) {
        hidden_layer(frag, kFragL2 + 32 * h, (const floatx4*)(bias + (h + 1) * kDH), l, g, Ba, Bb);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
#pragma unroll
            for (int c = 0; c < 4; ++c) Ba[nt][c] = Bb[nt][c];
        }
    }
    // output layer: one 16-row tile, row 0 is the output
    floatx4 o[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) o[nt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    bf16x8 an = frag[kFragL5 * 64 + l];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const bf16x8 a = an;
        if (c < 3) an = frag[(kFragL5 + c + 1) * 64 + l];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
            o[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, Ba[nt][c], o[nt], 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
    }
    // lane col of group 0 holds y of particle base + 16 nt + col in o[nt][0]
    const int rel = l - base;
    float y = 0.0f;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const float v = __shfl(o[nt][0], col, 64);
        if (rel >= 0 && (rel >> 4) == nt) y = v;
    }
    return y + bias[4 * kDH];
}

// y for all 64 particles of a wavefront (64 / (16 NT) passes of NT column tiles).
template <int NT>
__device__ __forceinline__ float mlp_wave(const bf16x8* __restrict__ frag, const float* __restrict__ bias,
                                          const float f[8]) {
    static_assert(NT == 2 || NT == 4, "passes of 32 or 64 particles");
    if (NT == 4) return mlp_pass<NT>(frag, bias, f, 0);
    const float y0 = mlp_pass<NT>(frag, bias, f, 0);
    const float y1 = mlp_pass<NT>(frag, bias, f, 32);
    return (threadIdx.x & 63) < 32 ? y0 : y1;
}

// log R of channel ch from the network output y and the normalised features f[0..3]
// (selects with constant indices: a runtime index into the by-value argument
// would put it in scratch memory)
__device__ __forceinline__ float pick(const float a[4], int ch) {
    return ch == 0 ? a[0] : (ch == 1 ? a[1] : (ch == 2 ? a[2] : a[3]));
}
__device__ __forceinline__ float log_rate(const MlpConst& mc, int ch, const float f[8], float y) {
    float v = pick(mc.out_mu, ch);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float li = ch == 0 ? mc.out_lin[0][i]
                                 : (ch == 1 ? mc.out_lin[1][i] : (ch == 2 ? mc.out_lin[2][i] : mc.out_lin[3][i]));
        v = fmaf(li, f[i], v);
    }
    return fmaf(pick(mc.out_sigma, ch), y, v);
}

// MODE 0: photons -> lambda_P; 1: axions -> thermal P_abs; 2: axions -> a->gamma mean.
// NT: 16-particle column tiles per network pass (64 particles per pass where the
// mode's registers allow it: every weight fragment then feeds four tiles).
template <typename T, int MODE, int NT>
__global__ void __launch_bounds__(kInfThreadsP)
k_rates_mlp(int64_t n, int ee_on, KParams kp, MlpConst mc, double g2P, double g2e,
            double boost,
            double lam_unit_P, double lam_unit_ag, const double* __restrict__ state,
            const float* __restrict__ p32, const double* __restrict__ p64, int32_t nion, double Zion,
            const T* __restrict__ w, const T* __restrict__ px, const T* __restrict__ py,
            const T* __restrict__ pz, const int32_t* __restrict__ cell,
            const unsigned char* __restrict__ blob, T* __restrict__ out,
            unsigned long long* __restrict__ nfallback) {
    __shared__ __align__(16) unsigned char lds[kBlobBytes];
    // weights to LDS once per workgroup (grid-stride over particle tiles below)
    {
        const uint4* src = (const uint4*)blob;
        uint4* dst = (uint4*)lds;
        for (int k = threadIdx.x; k < (int)(kBlobBytes / 16); k += blockDim.x) dst[k] = src[k];
    }
    __syncthreads();
    const bf16x8* frag = (const bf16x8*)lds;
    const float* bias = (const float*)(lds + (size_t)kNFrag * kFragBytes);
    const T* pref = PrefOf<T>::get(p32, p64);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t waves_total = (int64_t)gridDim.x * (kInfThreadsP / 64);
    const int64_t tiles = (n + 63) / 64;
    unsigned long long fb_count = 0;
    for (int64_t t = (int64_t)blockIdx.x * (kInfThreadsP / 64) + wave; t < tiles; t += waves_total) {
        const int64_t i = t * 64 + lane;
        const bool live = i < n;
        const int64_t ii = live ? i : n - 1;
        const int32_t c = cell[ii];
        // the network's inputs: only these stay live across the passes (the rest of the
        // particle and cell state is read again for the rate)
        float f[8];
        bool in_dom;
        {
            const double* st = state + (int64_t)c * AXPIC_STATE_N;
            const double Tc = st[0], ne = st[1], k2 = st[7];
            const double x = kMe * sqrt((double)psq<T>(px, py, pz, ii)) / Tc;
            in_dom = nion == 1 && (Zion == 1.0 || Zion == 2.0) && Tc >= mc.T_lo && Tc <= mc.T_hi &&
                     ne >= mc.ne_lo && ne <= mc.ne_hi && x >= mc.x_lo && x <= mc.x_hi;
            // the features in FP32 (they enter the network rounded to BF16): FP32 logarithms
            // of the FP64 state, the domain test above in FP64
            f[0] = (logf((float)x) - mc.feat_lo[0]) * mc.feat_sc[0] - 1.0f;
            f[1] = ((0.5f * logf((float)k2) - logf((float)Tc)) - mc.feat_lo[1]) * mc.feat_sc[1] - 1.0f;
            f[2] = (logf((float)ne) - mc.feat_lo[2]) * mc.feat_sc[2] - 1.0f;
            f[3] = ((float)Zion - mc.feat_lo[3]) * mc.feat_sc[3] - 1.0f;
        }
        // one network pass per channel: Primakoff (modes 0, 2) or the three thermal ones.
        // No memory access moves across a pass (the empty asm statements): what it would
        // carry through the pass does not fit the registers at 64 particles per pass.
        float y0 = 0.0f, y1 = 0.0f, y2 = 0.0f;
        constexpr int c0 = MODE == 1 ? 1 : 0, c1 = MODE == 1 ? 3 : 0;
#pragma unroll 1
        for (int ch = c0; ch <= c1; ++ch) {
            f[4] = ch == 0 ? 1.0f : 0.0f; f[5] = ch == 1 ? 1.0f : 0.0f;
            f[6] = ch == 2 ? 1.0f : 0.0f; f[7] = ch == 3 ? 1.0f : 0.0f;
            asm volatile("" ::: "memory");
            const float yy = mlp_wave<NT>(frag, bias, f);
            asm volatile("" ::: "memory");
            if (ch <= 1) y0 = yy;
            else if (ch == 2) y1 = yy;
            else y2 = yy;
        }
        const float y[3] = {y0, y1, y2};
        const double* st = state + (int64_t)c * AXPIC_STATE_N;
        const double Tc = st[0];
        const T* pc = pref + (int64_t)c * AXPIC_PREF_N;
        const T wt = w[ii];
        const T p2 = psq<T>(px, py, pz, ii);
        double res;
        if constexpr (MODE == 0 || MODE == 2) {
            const double GdtP = g2P * boost * exp((double)log_rate(mc, 0, f, y[0])) * kp.dt_phys;
            if constexpr (MODE == 0) {
                res = in_dom ? (double)wt * lam_unit_P * (-expm1(-GdtP))
                             : (double)lambda_primakoff<T>(pc, wt, p2);
            } else {
                res = in_dom ? (double)wt * lam_unit_ag * (-expm1(-kp.inv_ratio * GdtP))
                             : (double)lambda_ag<T>(kp, pc, wt, p2);
            }
        } else {
            double G = 0.0;
#pragma unroll
            for (int ch = 1; ch <= 3; ++ch) {
                const bool on = (ch == 1) ? (kp.channels & AXPIC_COMPTON) != 0
                                          : ((kp.channels & AXPIC_BREMS) != 0 && (ch == 2 || ee_on));
                // the brems targets exclude the cell's screening-fit factor; put it back
                const double supp = ch == 1 ? 1.0 : fmax(0.0, brems_suppression(Tc, st[5], st[6], ch == 3));
                if (on) G += supp * exp((double)log_rate(mc, ch, f, y[ch - 1]));
            }
            res = in_dom ? -expm1(-g2e * boost * G * kp.dt_phys)
                         : (double)pabs_thermal<T>(kp, pc, energy_keV(p2));
            if (!(wt > (T)0)) res = 0.0;
        }
        if (MODE != 1 && !(wt > (T)0)) res = 0.0;
        if (live) {
            out[i] = (T)res;
            fb_count += in_dom ? 0 : 1;
        }
    }
    for (int o = 32; o > 0; o >>= 1) fb_count += __shfl_xor(fb_count, o, 64);
    if (lane == 0 && fb_count && nfallback) atomicAdd(nfallback, fb_count);
}


// ------------------------------------------------------------------ per-cell tables
// Apart from omega, every input of the surrogate is constant in a cell, so the
// network can run once per (cell, node) on a grid in u = ln(omega/T) and the
// particles interpolate: the matrix-core work scales with cells x nodes.

// Row r = c nodes + j of the table: node u_j = u0 + j h of cell c.  Slot 0
// receives log R of the Primakoff conversion, slot 1 the log of the sum of the
// enabled thermal channels' absorption rates (brems times the cell's
// screening-fit factor; -inf if that sum is zero).  Cells outside the training
// box get NaN in the slots written.
__global__ void __launch_bounds__(kInfThreads)
k_mlp_table(int64_t ncell, int nodes, int slot0, int slot1, int c_on, int bz_on, int be_on,
            MlpConst mc, const double* __restrict__ state, int32_t nion, double Zion, double u0,
            double h, const unsigned char* __restrict__ blob, float* __restrict__ table) {
    __shared__ __align__(16) unsigned char lds[kBlobBytes];
    {
        const uint4* src = (const uint4*)blob;
        uint4* dst = (uint4*)lds;
        for (int k = threadIdx.x; k < (int)(kBlobBytes / 16); k += blockDim.x) dst[k] = src[k];
    }
    __syncthreads();
    const bf16x8* frag = (const bf16x8*)lds;
    const float* bias = (const float*)(lds + (size_t)kNFrag * kFragBytes);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t rows = ncell * nodes;
    const int64_t waves_total = (int64_t)gridDim.x * (kInfThreads / 64);
    const int64_t tiles = (rows + 63) / 64;
    for (int64_t t = (int64_t)blockIdx.x * (kInfThreads / 64) + wave; t < tiles; t += waves_total) {
        const int64_t r = t * 64 + lane;
        const bool live = r < rows;
        const int64_t rr = live ? r : rows - 1;
        const int64_t c = rr / nodes;
        const int j = (int)(rr - c * nodes);
        const double* st = state + c * AXPIC_STATE_N;
        const double Tc = st[0], ne = st[1], k2 = st[7];
        const bool in_box = nion == 1 && (Zion == 1.0 || Zion == 2.0) && Tc >= mc.T_lo &&
                            Tc <= mc.T_hi && ne >= mc.ne_lo && ne <= mc.ne_hi;
        float f[8];
        // FP32 logarithms of the FP64 state (the features enter the network as BF16)
        f[0] = ((float)(u0 + j * h) - mc.feat_lo[0]) * mc.feat_sc[0] - 1.0f;
        f[1] = ((0.5f * logf((float)k2) - logf((float)Tc)) - mc.feat_lo[1]) * mc.feat_sc[1] - 1.0f;
        f[2] = (logf((float)ne) - mc.feat_lo[2]) * mc.feat_sc[2] - 1.0f;
        f[3] = ((float)Zion - mc.feat_lo[3]) * mc.feat_sc[3] - 1.0f;
        float* out = table + c * 2 * nodes + j;
        if (slot0) {
            f[4] = 1.0f; f[5] = 0.0f; f[6] = 0.0f; f[7] = 0.0f;
            const float y = mlp_wave<kNTTable>(frag, bias, f);
            if (live) out[0] = in_box ? log_rate(mc, 0, f, y) : NAN;
        }
        if (slot1) {
            double G = 0.0;
#pragma unroll 1
            for (int ch = 1; ch <= 3; ++ch) {
                const int on = ch == 1 ? c_on : (ch == 2 ? bz_on : be_on);
                if (!on) continue;                           // uniform over the grid
                f[4] = 0.0f; f[5] = ch == 1 ? 1.0f : 0.0f; f[6] = ch == 2 ? 1.0f : 0.0f;
                f[7] = ch == 3 ? 1.0f : 0.0f;
                const float y = mlp_wave<kNTTable>(frag, bias, f);
                const double supp = ch == 1 ? 1.0 : fmax(0.0, brems_suppression(Tc, st[5], st[6], ch == 3));
                G += supp * exp((double)log_rate(mc, ch, f, y));
            }
            if (live) out[nodes] = in_box ? (float)log(G) : NAN;
        }
    }
}

// Per-particle rates from the tables: 4-point Lagrange interpolation in u on the
// nodes k .. k+3 around the particle, k = clamp(floor(t) - 1, 0, nodes - 4),
// t = (u - u0)/h, in FP64.  Modes as k_rates_mlp; particles outside
// [x_lo, x_hi] or in a cell without a table take the plain rate.
template <typename T>
__global__ void __launch_bounds__(256)
k_rates_table(int64_t n, int mode, int nodes, double u0, double h, double x_lo, double x_hi,
              KParams kp, double g2P, double g2e, double boost, double lam_unit_P,
              double lam_unit_ag, const double* __restrict__ state, const float* __restrict__ p32,
              const double* __restrict__ p64, const T* __restrict__ w, const T* __restrict__ px,
              const T* __restrict__ py, const T* __restrict__ pz, const int32_t* __restrict__ cell,
              const float* __restrict__ table, T* __restrict__ out,
              unsigned long long* __restrict__ nfallback) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool live = i < n;
    bool plain = false;
    if (live) {
        const int32_t c = cell[i];
        const double Tc = state[(int64_t)c * AXPIC_STATE_N];
        const T p2 = psq<T>(px, py, pz, i);
        const T wt = w[i];
        const double om = kMe * sqrt((double)p2);
        const double x = om / Tc;
        const float* row = table + ((int64_t)c * 2 + (mode == 1 ? 1 : 0)) * nodes;
        const float L0 = row[0];
        plain = isnan(L0) || !(x >= x_lo && x <= x_hi);
        double L = 0.0;
        if (!plain) {
            const double t = (log(x) - u0) / h;
            const int k = min(max((int)floor(t) - 1, 0), nodes - 4);
            const double s = t - k, a = s - 1.0, b = s - 2.0, d = s - 3.0;
            L = -(a * b * d) / 6.0 * row[k] + (s * b * d) / 2.0 * row[k + 1] -
                (s * a * d) / 2.0 * row[k + 2] + (s * a * b) / 6.0 * row[k + 3];
        }
        const T* pc = PrefOf<T>::get(p32, p64) + (int64_t)c * AXPIC_PREF_N;
        double res;
        if (mode == 0) {
            res = plain ? (double)lambda_primakoff<T>(pc, wt, p2)
                        : (double)wt * lam_unit_P * (-expm1(-g2P * boost * exp(L) * kp.dt_phys));
        } else if (mode == 2) {
            res = plain ? (double)lambda_ag<T>(kp, pc, wt, p2)
                        : (double)wt * lam_unit_ag *
                              (-expm1(-kp.inv_ratio * g2P * boost * exp(L) * kp.dt_phys));
        } else {
            res = plain ? (double)pabs_thermal<T>(kp, pc, energy_keV(p2))
                        : (L0 == -INFINITY ? 0.0 : -expm1(-g2e * boost * exp(L) * kp.dt_phys));
        }
        if (!(wt > (T)0)) res = 0.0;
        out[i] = (T)res;
    }
    const unsigned long long m = __ballot(live && plain);
    if ((threadIdx.x & 63) == 0 && m && nfallback) atomicAdd(nfallback, (unsigned long long)__popcll(m));
}

// ------------------------------------------------------------------ training samples
// Samples of the surrogate's target generated by the plain rates in FP64: one
// uniform cell per sample (electron density ne, ions of charge Z at density
// ne/Z with A = 1 for Z = 1 and A = 4 for Z = 2, temperature T), omega = x T,
// couplings 1: channel 0 Gamma_{gamma->a}/g^2 (Sec. II.F), channels 1-3 the
// detailed-balance absorption rate (eq. gamma_abs) of the Compton-like, e-Z
// and e-e channels per g_ae^2.
__global__ void __launch_bounds__(256)
k_surrogate_samples(int64_t n, axpic_params prm, const double* __restrict__ T,
                    const double* __restrict__ ne, const double* __restrict__ Z,
                    const double* __restrict__ x, const int32_t* __restrict__ ch,
                    double* __restrict__ feat, double* __restrict__ logR) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    axpic_params p = prm;
    p.g_agg_GeV = 1.0; p.g_ae = 1.0; p.boost = 1.0; p.quasi_neutral = 0; p.kappa_mode = 0;
    p.brems_ee = 1;
    const double Zi = Z[i], Ai = Zi == 1.0 ? 1.0 : 4.0, Ti = T[i], nei = ne[i];
    const double ni = nei / Zi;
    const double rho = ni * Ai * kMu;
    const LocalState L = local_state(Ti, nei, Zi * ni, Zi * Zi * ni, rho, Zi == 1.0 ? rho : 0.0, p);
    const double E = x[i] * Ti, xx = x[i];
    const double hc3 = kHbarcKeVcm * kHbarcKeVcm * kHbarcKeVcm;
    double R;
    if (ch[i] == 0) {
        R = L.G_P0 * screenF(4.0 * E * E / L.kappa2);
    } else if (ch[i] == 1) {
        const double aC = L.ne_dep * L.G_C * 2.0 * kPi * kPi * hc3 / (24.0 * kZeta5 * pow(Ti, 5.0));
        R = aC * E * E / (p.eq_stats ? -expm1(-xx) : 1.0);
    } else {
        const double k = p.brems_k, th = p.brems_theta;
        const double G = ch[i] == 2 ? L.G_BeZ : L.G_Bee;
        const double aB = L.ne_dep * G * 2.0 * kPi * kPi * hc3 / (exp(lgamma(k)) * pow(th, k) * Ti * Ti * Ti);
        const double shape = p.eq_stats ? exp(xx * (1.0 - 1.0 / th)) : exp(-xx / th) * expm1(xx);
        R = aB * exp((k - 3.0) * log(xx)) * shape;
        const double supp = brems_suppression(Ti, L.rho, L.XH, ch[i] == 3);
        R = supp > 0.0 ? R / supp : __builtin_nan("");
    }
    logR[i] = log(R);
    feat[4 * i + 0] = log(xx);
    feat[4 * i + 1] = 0.5 * log(L.kappa2) - log(Ti);
    feat[4 * i + 2] = log(nei);
    feat[4 * i + 3] = Zi;
}

KParams kparams_for(const axpic_grid* g, const axpic_params* prm, double w_ref_g) {
    KParams k;
    std::memset(&k, 0, sizeof(k));
    k.dt_phys = g->dt / g->omega0;
    k.w_a = prm->w_a;
    for (int i = 0; i < 3; ++i) k.wa_mul[i] = prm->wa_mul[i];
    k.w_gamma_prod = prm->w_gamma_prod > 0.0 ? prm->w_gamma_prod : w_ref_g;
    k.inv_ratio = prm->prim_inv_ratio;
    k.ag_unit = (w_ref_g > 0.0 && k.w_gamma_prod > 0.0)
                    ? prm->prim_inv_ratio * prm->w_a * prm->w_a * prm->wa_mul[0] /
                          (w_ref_g * k.w_gamma_prod)
                    : 0.0;
    k.brems_k = prm->brems_k;
    k.brems_theta = prm->brems_theta;
    k.brems_km3 = prm->brems_k - 3.0;
    k.brems_c1 = 1.0 - 1.0 / prm->brems_theta;
    k.channels = prm->channels;
    k.inverse = prm->inverse;
    k.eq_stats = prm->eq_stats;
    return k;
}

}  // namespace

extern "C" {

size_t axpic_mlp_blob_bytes(void) { return kBlobBytes; }

size_t axpic_mlp_train_ws_bytes(int64_t batch) {
    // Z1..Z4, H1..H4 [B][128], Z5 [B][32], dZ [B][128], dH [B][128], grads, split-K partials
    return sizeof(float) * (size_t)batch * (8 * kDH + kD5 + 2 * kDH) + sizeof(float) * kNParams +
           sizeof(float) * (size_t)kSplitMax * kDH * kDH;
}

axpic_status axpic_surrogate_samples(const axpic_params* prm, int64_t n, const double* T,
                                     const double* ne, const double* Z, const double* x,
                                     const int32_t* ch, double* feat, double* logR, void* stream) {
    if (!prm || n < 0 || (n && (!T || !ne || !Z || !x || !ch || !feat || !logR))) return AXPIC_E_INVAL;
    if (n == 0) return AXPIC_OK;
    LAUNCH("k_surrogate_samples", k_surrogate_samples, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       S(stream), n, *prm, T, ne, Z, x, ch, feat, logR);
    return launched();
}

size_t axpic_mlp_prepare_ws_bytes(void) {
    return sizeof(double) * ((size_t)kPrepBlocks * kMomN + 4 * kMomN + 8);
}

// Gaussian elimination with partial pivoting of the 5 x 5 normal equations.
static bool solve5(double A[5][5], double b[5], double x[5]) {
    for (int c = 0; c < 5; ++c) {
        int piv = c;
        for (int r = c + 1; r < 5; ++r)
            if (std::fabs(A[r][c]) > std::fabs(A[piv][c])) piv = r;
        if (!(std::fabs(A[piv][c]) > 0.0)) return false;
        if (piv != c) {
            for (int k = 0; k < 5; ++k) std::swap(A[c][k], A[piv][k]);
            std::swap(b[c], b[piv]);
        }
        for (int r = c + 1; r < 5; ++r) {
            const double f = A[r][c] / A[c][c];
            for (int k = c; k < 5; ++k) A[r][k] -= f * A[c][k];
            b[r] -= f * b[c];
        }
    }
    for (int r = 4; r >= 0; --r) {
        double v = b[r];
        for (int k = r + 1; k < 5; ++k) v -= A[r][k] * x[k];
        x[r] = v / A[r][r];
    }
    return true;
}

static PrepNorm to_prep(const axpic_mlp_norm* nm) {
    PrepNorm p;
    for (int k = 0; k < 4; ++k) {
        p.lo[k] = nm->lo[k]; p.sc[k] = nm->sc[k]; p.mu[k] = nm->mu[k]; p.sigma[k] = nm->sigma[k];
        for (int j = 0; j < 4; ++j) p.lin[k][j] = nm->lin[k][j];
    }
    return p;
}

axpic_status axpic_mlp_prepare(const double* feat, const double* logR, const int32_t* ch, int64_t n,
                               void* ws, size_t ws_bytes, axpic_mlp_norm* norm, void* stream) {
    if (!norm || n < 1 || !feat || !logR || !ch || !ws || ws_bytes < axpic_mlp_prepare_ws_bytes())
        return AXPIC_E_INVAL;
    hipStream_t s = S(stream);
    double* part = (double*)ws;
    double* out = part + (size_t)kPrepBlocks * kMomN;
    double h[4 * kMomN];
    // feature ranges over the valid rows (Z spans [1, 2])
    LAUNCH("k_prep_range", k_prep_range, dim3(kPrepBlocks), dim3(256), 0, s, n, feat, logR, part);
    LAUNCH("k_prep_sum", k_prep_sum, dim3(1), dim3(64), 0, s, kPrepBlocks, 6, part, out, 1);
    if (hipMemcpyAsync(h, out, sizeof(double) * 6, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return AXPIC_E_DEVICE;
    std::memset(norm, 0, sizeof(*norm));
    for (int k = 0; k < 3; ++k) {
        if (!(h[3 + k] > h[k])) return AXPIC_E_DOMAIN;
        norm->lo[k] = h[k];
        norm->sc[k] = 2.0 / (h[3 + k] - h[k]);
    }
    norm->lo[3] = 1.0; norm->sc[3] = 2.0;
    const PrepNorm pn = to_prep(norm);
    for (int c = 0; c < 4; ++c) {
        LAUNCH("k_prep_moments", k_prep_moments, dim3(kPrepBlocks), dim3(256), 0, s, n, feat, logR,
               ch, c, pn, part);
        LAUNCH("k_prep_sum", k_prep_sum, dim3(1), dim3(64), 0, s, kPrepBlocks, kMomN, part,
               out + c * kMomN, 0);
    }
    if (hipMemcpyAsync(h, out, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return AXPIC_E_DEVICE;
    for (int c = 0; c < 4; ++c) {
        const double* m = h + c * kMomN;
        double A[5][5], r[5], x[5];
        int q = 0;
        for (int a = 0; a < 5; ++a)
            for (int b = a; b < 5; ++b) { A[a][b] = A[b][a] = m[q]; ++q; }
        for (int a = 0; a < 5; ++a) r[a] = m[15 + a];
        const double cnt = A[0][0];
        norm->count[c] = (int64_t)std::llround(cnt);
        if (!(cnt > 5.0)) return AXPIC_E_DOMAIN;
        double Ac[5][5], rc[5];
        std::memcpy(Ac, A, sizeof(A)); std::memcpy(rc, r, sizeof(r));
        if (!solve5(Ac, rc, x)) return AXPIC_E_DOMAIN;
        norm->mu[c] = x[0];
        for (int k = 0; k < 4; ++k) norm->lin[c][k] = x[1 + k];
        // residual e = y - d.x: sum e = r0 - A0.x, sum e^2 = yy - 2 x.r + x.A.x
        double se = r[0], see = m[20];
        for (int a = 0; a < 5; ++a) {
            se -= A[0][a] * x[a];
            see -= 2.0 * x[a] * r[a];
            for (int b = 0; b < 5; ++b) see += x[a] * A[a][b] * x[b];
        }
        const double var = (see - se * se / cnt) / (cnt - 1.0);
        // a channel that the affine fit reproduces keeps a residual of rounding noise
        // only: the floor keeps the network from fitting it
        norm->sigma[c] = std::max(var > 0.0 ? std::sqrt(var) : 0.0, 1e-3);
    }
    return AXPIC_OK;
}

axpic_status axpic_mlp_design(const double* feat, const double* logR, const int32_t* ch, int64_t n,
                              const axpic_mlp_norm* norm, float* X, float* Y, void* stream) {
    if (!norm || n < 0 || (n && (!feat || !logR || !ch || !X || !Y))) return AXPIC_E_INVAL;
    if (((uintptr_t)X & 15u) != 0) return AXPIC_E_INVAL;
    if (n == 0) return AXPIC_OK;
    LAUNCH("k_prep_design", k_prep_design, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, S(stream),
           n, feat, logR, ch, to_prep(norm), X, Y);
    return launched();
}

axpic_status axpic_mlp_batch(const float* X, const float* Y, int64_t n, int64_t batch, uint64_t seed,
                             int64_t step, float* Xb, float* Yb, void* stream) {
    if (n < 1 || n > 0xFFFFFFFFll || batch < 1 || !X || !Y || !Xb || !Yb) return AXPIC_E_INVAL;
    if ((((uintptr_t)X | (uintptr_t)Xb) & 15u) != 0) return AXPIC_E_INVAL;
    LAUNCH("k_prep_batch", k_prep_batch, dim3((unsigned)((batch + 255) / 256)), dim3(256), 0,
           S(stream), n, X, Y, batch, (uint32_t)seed, (uint32_t)(seed >> 32), step, Xb, Yb);
    return launched();
}

axpic_status axpic_mlp_pack(const float* master, void* blob, void* stream) {
    if (!master || !blob) return AXPIC_E_INVAL;
    LAUNCH("k_mlp_pack", k_mlp_pack, dim3(kNFrag), dim3(64), 0, S(stream), master, (__bf16*)blob,
                       (float*)((unsigned char*)blob + (size_t)kNFrag * kFragBytes));
    return launched();
}

// Long K (the weight gradients, K = batch) is split so that the grid fills the chip; the
// partial tiles go to `part` (kSplitMax M N floats) and are summed in split order.
static void gemm(int prec, int64_t M, int64_t N, int64_t K, const float* A, int64_t lda, int tA,
                 const float* B, int64_t ldb, int tB, float* C, int64_t ldc, const float* bias,
                 float* part, hipStream_t s) {
    if (prec == AXPIC_MLP_F32) {
        LAUNCH("k_gemm_f32", k_gemm_f32, dim3((unsigned)(N / 16), (unsigned)(M / 16)), dim3(256), 0,
               s, M, N, K, A, lda, tA, B, ldb, tB, C, ldc, bias);
        return;
    }
    const int64_t tiles = (M / 32) * (N / 32);
    int split = 1;
    while (split < kSplitMax && tiles * split < 256 && K % (64 * split) == 0) split *= 2;
    LAUNCH("k_gemm_bf16", k_gemm_bf16, dim3((unsigned)(N / 32), (unsigned)(M / 32), (unsigned)split),
           dim3(256), 0, s, M, N, K, A, lda, tA, B, ldb, tB, split > 1 ? part : C, ldc, bias);
    if (split > 1)
        LAUNCH("k_gemm_splitk_sum", k_gemm_splitk_sum, dim3((unsigned)((M * N + 255) / 256)),
               dim3(256), 0, s, M, N, split, (const float*)part, C, ldc, bias);
}

struct TrainWs {
    float *Z[6], *H[5], *dZ, *dH, *grad, *part;
};

static TrainWs carve_train(void* ws, int64_t Bn) {
    TrainWs t;
    float* p = (float*)ws;
    t.H[0] = nullptr;
    for (int l = 1; l <= 4; ++l) { t.Z[l] = p; p += Bn * kDH; }
    for (int l = 1; l <= 4; ++l) { t.H[l] = p; p += Bn * kDH; }
    t.Z[5] = p; p += Bn * kD5;
    t.dZ = p; p += Bn * kDH;
    t.dH = p; p += Bn * kDH;
    t.grad = p; p += kNParams;
    t.part = p;
    return t;
}

/* Forward pass with saved activations (training layout): X [B][32] (features in
 * columns 0..7), y[b] = Z5[b][0]. */
axpic_status axpic_mlp_forward(const float* master, const float* X, int64_t batch, int32_t precision,
                               void* ws, size_t ws_bytes, float* y, void* stream) {
    if (!master || !X || !ws || batch <= 0 || batch % 32 || ws_bytes < axpic_mlp_train_ws_bytes(batch))
        return AXPIC_E_INVAL;
    if (precision != AXPIC_MLP_BF16 && precision != AXPIC_MLP_F32) return AXPIC_E_INVAL;
    hipStream_t s = S(stream);
    TrainWs t = carve_train(ws, batch);
    const float* hin = X;
    for (int l = 1; l <= 5; ++l) {
        gemm(precision, batch, dOut(l), dIn(l), hin, dIn(l), 0, master + offW(l), dOut(l), 0, t.Z[l],
             dOut(l), master + offB(l), t.part, s);
        if (l <= 4) {
            const int64_t n = batch * kDH;
            LAUNCH("k_act_fwd", k_act_fwd, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n,
                               t.Z[l], t.H[l]);
            hin = t.H[l];
        }
    }
    if (y)
        LAUNCH("k_col0", k_col0, dim3((unsigned)((batch + 255) / 256)), dim3(256), 0, s, batch,
                           t.Z[5], y);
    return launched();
}

/* Mean-squared-error loss and its gradient with respect to the FP32 master
 * parameters (padded layout, AXPIC_MLP_PARAMS floats) for a batch X, Y. */
axpic_status axpic_mlp_loss_grad(const float* master, const float* X, const float* Y, int64_t batch,
                                 int32_t precision, void* ws, size_t ws_bytes, float* grad,
                                 double* loss, void* stream) {
    if (!Y || !grad) return AXPIC_E_INVAL;
    axpic_status st = axpic_mlp_forward(master, X, batch, precision, ws, ws_bytes, nullptr, stream);
    if (st != AXPIC_OK) return st;
    hipStream_t s = S(stream);
    TrainWs t = carve_train(ws, batch);
    if (loss) LAUNCH("k_zero_d", k_zero_d, dim3(1), dim3(64), 0, s, loss);
    float* dZ5 = t.dH;   // [B][32] fits in dH
    LAUNCH("k_mse_grad", k_mse_grad, dim3((unsigned)((batch + 255) / 256)), dim3(256), 0, s, batch,
                       t.Z[5], Y, dZ5, loss);
    const float* dZ = dZ5;
    for (int l = 5; l >= 1; --l) {
        const float* hin = l == 1 ? X : t.H[l - 1];
        // weight gradient: hin^T dZ
        gemm(precision, dIn(l), dOut(l), batch, hin, dIn(l), 1, dZ, dOut(l), 0, grad + offW(l),
             dOut(l), nullptr, t.part, s);
        LAUNCH("k_colsum", k_colsum, dim3((unsigned)dOut(l)), dim3(256), 0, s, batch,
                           (int64_t)dOut(l), dZ, grad + offB(l));
        if (l == 1) break;
        // dH_{l-1} = dZ W^T, then through the activation
        float* dst = (dZ == t.dZ) ? t.dH : t.dZ;
        gemm(precision, batch, dIn(l), dOut(l), dZ, dOut(l), 0, master + offW(l), dOut(l), 1, dst,
             dIn(l), nullptr, t.part, s);
        const int64_t n = batch * kDH;
        LAUNCH("k_act_bwd", k_act_bwd, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n,
                           t.Z[l - 1], dst);
        dZ = dst;
    }
    return launched();
}

axpic_status axpic_mlp_adam(float* master, const float* grad, float* m, float* v, int64_t step,
                            float lr, float beta1, float beta2, float eps, void* stream) {
    if (!master || !grad || !m || !v || step < 1) return AXPIC_E_INVAL;
    const float c1 = 1.0f - powf(beta1, (float)step), c2 = 1.0f - powf(beta2, (float)step);
    LAUNCH("k_adam", k_adam, dim3((unsigned)((kNParams + 255) / 256)), dim3(256), 0, S(stream),
                       (int64_t)kNParams, master, grad, m, v, lr, beta1, beta2, eps, c1, c2);
    return launched();
}

static MlpConst mlp_const(const axpic_mlp* net) {
    MlpConst mc;
    for (int i = 0; i < 4; ++i) {
        mc.feat_lo[i] = net->feat_lo[i]; mc.feat_sc[i] = net->feat_sc[i];
        mc.out_mu[i] = net->out_mu[i]; mc.out_sigma[i] = net->out_sigma[i];
        for (int j = 0; j < 4; ++j) mc.out_lin[i][j] = net->out_lin[i][j];
    }
    mc.T_lo = net->T_lo; mc.T_hi = net->T_hi; mc.ne_lo = net->ne_lo; mc.ne_hi = net->ne_hi;
    mc.x_lo = net->x_lo; mc.x_hi = net->x_hi;
    return mc;
}

static int compute_units() {
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            ncu = v;
    }
    return ncu;
}

axpic_status axpic_rates_mlp(const axpic_grid* g, const axpic_cells* cells, const axpic_params* prm,
                             const axpic_species* sp, int32_t channel, const axpic_mlp* net,
                             void* out, unsigned long long* n_fallback, void* stream) {
    if (prm && prm->m_a_keV != 0.0) return AXPIC_E_UNSUPPORTED;   // the surrogate is massless
    if (!g || !cells || !prm || !sp || !net || !net->blob || (!out && sp->n)) return AXPIC_E_INVAL;
    if (sp->n < 0 || (sp->n && (!sp->w || !sp->cell || !sp->p[0] || !sp->p[1] || !sp->p[2])))
        return AXPIC_E_INVAL;
    if (!cells->state || !cells->pref32 || !cells->pref64) return AXPIC_E_INVAL;
    int mode;
    if (sp->kind == AXPIC_PHOTON && channel == AXPIC_PRIMAKOFF) mode = 0;
    else if (sp->kind == AXPIC_AXION && channel == (AXPIC_COMPTON | AXPIC_BREMS)) mode = 1;
    else if (sp->kind == AXPIC_AXION && channel == AXPIC_PRIMAKOFF) mode = 2;
    else return AXPIC_E_INVAL;
    if (sp->n == 0) return AXPIC_OK;
    KParams kp = kparams_for(g, prm, cells->w_ref_g);
    const MlpConst mc = mlp_const(net);
    const double g2P = prm->g_agg_GeV * prm->g_agg_GeV, g2e = prm->g_ae * prm->g_ae;
    const double lam_unit_P = cells->w_ref_g / (prm->w_a * prm->wa_mul[0]);
    const double lam_unit_ag = prm->w_a / kp.w_gamma_prod;
    const int ncu = compute_units();
    const int64_t tiles = (sp->n + 63) / 64;
    constexpr int kWaves = kInfThreadsP / 64;
    const int64_t wgs = std::min<int64_t>((tiles + kWaves - 1) / kWaves, (int64_t)ncu);
    const double Z = cells->nion == 1 ? cells->Zion[0] : 0.0;
    // 64 particles per network pass where the registers allow it (FP32), else 32
#define AXPIC_RATES_MLP(TT, MD, NT)                                                              \
    LAUNCH("k_rates_mlp", (k_rates_mlp<TT, MD, NT>), dim3((unsigned)wgs), dim3(kInfThreadsP), 0,   \
           S(stream), sp->n, prm->brems_ee, kp, mc, g2P, g2e, prm->boost, lam_unit_P, lam_unit_ag, \
           cells->state, cells->pref32, cells->pref64, cells->nion, Z, (const TT*)sp->w,           \
           (const TT*)sp->p[0], (const TT*)sp->p[1], (const TT*)sp->p[2], sp->cell,                \
           (const unsigned char*)net->blob, (TT*)out, n_fallback)
    if (sp->dtype == AXPIC_F32) {
        if (mode == 0) AXPIC_RATES_MLP(float, 0, 4);
        else if (mode == 1) AXPIC_RATES_MLP(float, 1, 4);
        else AXPIC_RATES_MLP(float, 2, 4);
    } else {
        if (mode == 0) AXPIC_RATES_MLP(double, 0, 2);
        else if (mode == 1) AXPIC_RATES_MLP(double, 1, 2);
        else AXPIC_RATES_MLP(double, 2, 2);
    }
#undef AXPIC_RATES_MLP
    return launched();
}

axpic_status axpic_mlp_table(const axpic_grid* g, const axpic_cells* cells, const axpic_params* prm,
                             int32_t channel, const axpic_mlp* net, int32_t nodes, double x_lo,
                             double x_hi, float* table, void* stream) {
    if (prm && prm->m_a_keV != 0.0) return AXPIC_E_UNSUPPORTED;   // the surrogate is massless
    if (!g || !cells || !prm || !net || !net->blob || !table) return AXPIC_E_INVAL;
    if (nodes < 4 || nodes > AXPIC_TAB_MAX_NODES || !(x_lo > 0.0) || !(x_hi > x_lo) ||
        !(x_lo >= net->x_lo) || !(x_hi <= net->x_hi))
        return AXPIC_E_INVAL;
    if (cells->ncell < 0 || (cells->ncell && !cells->state)) return AXPIC_E_INVAL;
    const int slot0 = (channel & AXPIC_PRIMAKOFF) != 0;
    const int slot1 = (channel & (AXPIC_COMPTON | AXPIC_BREMS)) != 0;
    if (!slot0 && !slot1) return AXPIC_E_INVAL;
    if (cells->ncell == 0) return AXPIC_OK;
    const int c_on = (prm->channels & AXPIC_COMPTON) != 0;
    const int bz_on = (prm->channels & AXPIC_BREMS) != 0;
    const int be_on = bz_on && prm->brems_ee;
    const double u0 = log(x_lo), h = (log(x_hi) - u0) / (nodes - 1);
    const int64_t tiles = (cells->ncell * nodes + 63) / 64;
    constexpr int kWaves = kInfThreads / 64;
    const int64_t wgs = std::min<int64_t>((tiles + kWaves - 1) / kWaves, (int64_t)compute_units());
    const double Z = cells->nion == 1 ? cells->Zion[0] : 0.0;
    LAUNCH("k_mlp_table", k_mlp_table, dim3((unsigned)wgs), dim3(kInfThreads), 0, S(stream),
           cells->ncell, (int)nodes, slot0, slot1, c_on, bz_on, be_on, mlp_const(net), cells->state,
           cells->nion, Z, u0, h, (const unsigned char*)net->blob, table);
    return launched();
}

axpic_status axpic_rates_table(const axpic_grid* g, const axpic_cells* cells, const axpic_params* prm,
                               const axpic_species* sp, int32_t channel, int32_t nodes, double x_lo,
                               double x_hi, const float* table, void* out,
                               unsigned long long* n_fallback, void* stream) {
    if (prm && prm->m_a_keV != 0.0) return AXPIC_E_UNSUPPORTED;   // the surrogate is massless
    if (!g || !cells || !prm || !sp || !table || (!out && sp->n)) return AXPIC_E_INVAL;
    if (nodes < 4 || nodes > AXPIC_TAB_MAX_NODES || !(x_lo > 0.0) || !(x_hi > x_lo))
        return AXPIC_E_INVAL;
    if (sp->n < 0 || (sp->n && (!sp->w || !sp->cell || !sp->p[0] || !sp->p[1] || !sp->p[2])))
        return AXPIC_E_INVAL;
    if (!cells->state || !cells->pref32 || !cells->pref64) return AXPIC_E_INVAL;
    int mode;
    if (sp->kind == AXPIC_PHOTON && channel == AXPIC_PRIMAKOFF) mode = 0;
    else if (sp->kind == AXPIC_AXION && channel == (AXPIC_COMPTON | AXPIC_BREMS)) mode = 1;
    else if (sp->kind == AXPIC_AXION && channel == AXPIC_PRIMAKOFF) mode = 2;
    else return AXPIC_E_INVAL;
    if (sp->n == 0) return AXPIC_OK;
    KParams kp = kparams_for(g, prm, cells->w_ref_g);
    const double g2P = prm->g_agg_GeV * prm->g_agg_GeV, g2e = prm->g_ae * prm->g_ae;
    const double lam_unit_P = cells->w_ref_g / (prm->w_a * prm->wa_mul[0]);
    const double lam_unit_ag = prm->w_a / kp.w_gamma_prod;
    const double u0 = log(x_lo), h = (log(x_hi) - u0) / (nodes - 1);
    const unsigned blocks = (unsigned)((sp->n + 255) / 256);
    if (sp->dtype == AXPIC_F32)
        LAUNCH("k_rates_table", k_rates_table<float>, dim3(blocks), dim3(256), 0, S(stream), sp->n,
               mode, (int)nodes, u0, h, x_lo, x_hi, kp, g2P, g2e, prm->boost, lam_unit_P,
               lam_unit_ag, cells->state, cells->pref32, cells->pref64, (const float*)sp->w,
               (const float*)sp->p[0], (const float*)sp->p[1], (const float*)sp->p[2], sp->cell,
               table, (float*)out, n_fallback);
    else
        LAUNCH("k_rates_table", k_rates_table<double>, dim3(blocks), dim3(256), 0, S(stream), sp->n,
               mode, (int)nodes, u0, h, x_lo, x_hi, kp, g2P, g2e, prm->boost, lam_unit_P,
               lam_unit_ag, cells->state, cells->pref32, cells->pref64, (const double*)sp->w,
               (const double*)sp->p[0], (const double*)sp->p[1], (const double*)sp->p[2], sp->cell,
               table, (double*)out, n_fallback);
    return launched();
}

}  // extern "C"
