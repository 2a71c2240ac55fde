// Learned angle proposal: a 64 -> 256 -> 256 -> 256 -> 256 MLP with GELU,
// BF16 weights and activations, FP32 accumulation on gfx950 matrix cores.
//
// Every matrix product goes through one tiled kernel: 64 x 64 output tiles,
// four waves per block, each wave a 32 x 32 quadrant built from
// v_mfma_f32_32x32x16_bf16 over K steps of 32 staged in LDS.  Operand
// layouts per lane (wave64): A row = lane % 32, k = 8 (lane / 32) .. +8;
// B column = lane % 32, same k; the 16 accumulators of a lane hold column
// lane % 32, rows 8 (j / 4) + 4 (lane / 32) + j % 4.  Epilogues fuse the
// bias, GELU and the GELU derivative so activations are written once.
//
// Rounding points (mirrored by the FP64 reference): inputs, weights, hidden
// activations after GELU and pre-activation gradients are BF16; products
// accumulate in FP32; master weights and Adam moments are FP32.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mlp_internal.h"

namespace dock {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint16_t f2bf(float f) {
  // round to nearest even
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Two FP32 values to packed BF16 (lo in the low half) in one instruction.
// For finite inputs it rounds to nearest even exactly like f2bf (checked on
// every finite value of a 3.4 M-value sweep including all-tie patterns);
// NaNs come out quieted rather than truncated.
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
  uint32_t r;
  asm("v_cvt_pk_bf16_f32 %0, %1, %2" : "=v"(r) : "v"(lo), "v"(hi));
  return r;
}

// erf by Abramowitz & Stegun 7.1.26: 1 - (a1 t + ... + a5 t^5) exp(-x^2),
// t = 1 / (1 + p |x|), odd in x; absolute error below 1.5e-7, far below the
// BF16 resolution of the activations it feeds.  Branch-free: one reciprocal
// and one exponential.
__device__ __forceinline__ float erf_as(float x) {
  const float ax = fabsf(x);
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, ax, 1.0f));
  float p = fmaf(1.061405429f, t, -1.453152027f);
  p = fmaf(p, t, 1.421413741f);
  p = fmaf(p, t, -0.284496736f);
  p = fmaf(p, t, 0.254829592f);
  p *= t;
  const float r = fmaf(-p, __expf(-ax * ax), 1.0f);
  return copysignf(r, x);
}

__device__ __forceinline__ float gelu_f(float z) {
  return 0.5f * z * (1.0f + erf_as(z * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad_f(float z) {
  return 0.5f * (1.0f + erf_as(z * 0.70710678118654752f)) +
         z * __expf(-0.5f * z * z) * 0.39894228040143268f;
}

constexpr int kTile = 64;  // output tile edge
constexpr int kKs = 32;    // K step staged in LDS

// C[m][n] = sum_k opA[m][k] * opB[k][n]
//   opA[m][k] = TA ? A[k * lda + m] : A[m * lda + k]
//   opB[k][n] = TB ? B[n * ldb + k] : B[k * ldb + n]
// K range [k0, k1) (split-K); M, N, K multiples of 64 / 64 / 32.
template <bool TA, bool TB, int EPI>
__global__ void __launch_bounds__(256) gemm_bf16_kernel(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) uint16_t sA[kTile][kKs + 8];  // [m][k]
  __shared__ __attribute__((aligned(16))) uint16_t sB[kTile][kKs + 8];  // [n][k]
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int m0 = blockIdx.y * kTile, n0 = blockIdx.x * kTile;
  const int split = blockIdx.z;
  const int kb = g.k_per_split * split, ke = kb + g.k_per_split;
  const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;
  f32x16 acc;
#pragma unroll
  for (int j = 0; j < 16; ++j) acc[j] = 0.0f;

  for (int k0 = kb; k0 < ke; k0 += kKs) {
    // stage A tile: 64 x 32
    if (!TA) {  // rows of 32 contiguous k: thread -> (row, 8-wide chunk)
      const int r = tid >> 2, c = (tid & 3) * 8;
      const uint4 v = *(const uint4 *)(g.A + (size_t)(m0 + r) * g.lda + k0 + c);
      *(uint4 *)&sA[r][c] = v;
    } else {  // storage [k][m]: 32 rows of 64 contiguous m
      const int kr = tid >> 3, c = (tid & 7) * 8;
      const uint4 v = *(const uint4 *)(g.A + (size_t)(k0 + kr) * g.lda + m0 + c);
      const uint16_t *e = (const uint16_t *)&v;
#pragma unroll
      for (int q = 0; q < 8; ++q) sA[c + q][kr] = e[q];
    }
    if (TB) {  // storage [n][k]
      const int r = tid >> 2, c = (tid & 3) * 8;
      const uint4 v = *(const uint4 *)(g.B + (size_t)(n0 + r) * g.ldb + k0 + c);
      *(uint4 *)&sB[r][c] = v;
    } else {  // storage [k][n]
      const int kr = tid >> 3, c = (tid & 7) * 8;
      const uint4 v = *(const uint4 *)(g.B + (size_t)(k0 + kr) * g.ldb + n0 + c);
      const uint16_t *e = (const uint16_t *)&v;
#pragma unroll
      for (int q = 0; q < 8; ++q) sB[c + q][kr] = e[q];
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kKs; kk += 16) {
      const int koff = kk + (lane >> 5) * 8;
      const bf16x8 a = *(const bf16x8 *)&sA[wm + (lane & 31)][koff];
      const bf16x8 b = *(const bf16x8 *)&sB[wn + (lane & 31)][koff];
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }

  const int col = n0 + wn + (lane & 31);
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int row = m0 + wm + (j >> 2) * 8 + (lane >> 5) * 4 + (j & 3);
    const size_t at = (size_t)row * g.ldc + col;
    float v = acc[j];
    if (EPI == kEpiStore) {
      g.Cf[(size_t)split * g.split_stride + at] = v;
    } else if (EPI == kEpiBiasGelu) {
      v += g.bias[col];
      g.Cf[at] = v;                    // pre-activation, kept for the backward pass
      g.Cb[at] = f2bf(gelu_f(v));      // activation, BF16
    } else if (EPI == kEpiBias) {
      g.Cf[at] = v + g.bias[col];
    } else if (EPI == kEpiGeluGrad) {  // dZ_prev = bf16(dA * gelu'(Z_prev))
      g.Cb[at] = f2bf(v * gelu_grad_f(g.aux[at]));
    }
  }
}

template <bool TA, bool TB, int EPI>
static hipError_t gemm_t(const GemmArgs &g, int M, int N, int splits, hipStream_t st) {
  hipLaunchKernelGGL((gemm_bf16_kernel<TA, TB, EPI>), dim3(N / kTile, M / kTile, splits),
                     dim3(256), 0, st, g);
  return hipGetLastError();
}

hipError_t gemm_bf16(const GemmArgs &g, bool ta, bool tb, int epi, int M, int N, int splits,
                     hipStream_t st) {
  if (M % kTile || N % kTile || g.k_per_split % kKs || splits < 1) return hipErrorInvalidValue;
#define DOCK_GEMM(TA, TB, E) \
  if (ta == TA && tb == TB && epi == E) return gemm_t<TA, TB, E>(g, M, N, splits, st);
  DOCK_GEMM(false, true, kEpiBiasGelu)
  DOCK_GEMM(false, true, kEpiBias)
  DOCK_GEMM(false, true, kEpiStore)
  DOCK_GEMM(false, false, kEpiGeluGrad)
  DOCK_GEMM(true, false, kEpiStore)
#undef DOCK_GEMM
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------- fused inference
// Forward pass of 64 rows per block through all four layers.  Activations
// stay in LDS (BF16, 64 x 256); each wave owns 64 output features (2 x 2
// tiles of 32 x 32) and reads its weight rows straight from global memory
// (L2-resident, stored [out][in] so the 8 k-values of an MFMA operand are
// contiguous).  The weights are the A operand and the activations the B
// operand, so a lane's accumulators hold runs of 4 consecutive output
// features of one row: the epilogue adds the bias and stores them as one
// 8-byte write (the next layer's k direction).  Arithmetic and rounding
// points are those of the tiled path: FP32 accumulation, bias, GELU, BF16
// activations; FP32 output.
constexpr int kInfRows = 64;
constexpr int kActPad = 8;

// Two blocks per CU (two waves per SIMD, within 256 registers and no spills):
// one block's GELU epilogue overlaps the other's matrix products.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
    mlp_infer_kernel(const uint16_t *x, const uint16_t *wb, const float *bias_src, float *y) {
  __shared__ __attribute__((aligned(16))) uint16_t sH[kInfRows][256 + kActPad];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const size_t row0 = (size_t)blockIdx.x * kInfRows;
  // input rows: 64 x 64 BF16
  for (int e = tid; e < kInfRows * 8; e += 256) {
    const int r = e >> 3, c = (e & 7) * 8;
    *(uint4 *)&sH[r][c] = *(const uint4 *)(x + (row0 + r) * 64 + c);
  }
  __syncthreads();
  const int kin[4] = {64, 256, 256, 256};
  const int64_t woff[4] = {kMlpW1, kMlpW2, kMlpW3, kMlpW4};
  const int64_t boff[4] = {kMlpB1, kMlpB2, kMlpB3, kMlpB4};
  const int col0 = wv * 64;
#pragma unroll 1
  for (int l = 0; l < 4; ++l) {
    f32x16 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int j = 0; j < 16; ++j) acc[a][b][j] = 0.0f;
    const uint16_t *W = wb + woff[l];
    const int K = kin[l];  // 64 or 256: a multiple of 4 k-steps of 16
    // Weight operands come from global memory (L2): they are fetched four
    // k-steps ahead into four rotating register sets, so the MFMAs of a step
    // do not wait for its loads.
    auto load_w = [&](int k0, bf16x8(&bo)[2]) {
      const int kk = k0 + (lane >> 5) * 8;
#pragma unroll
      for (int b = 0; b < 2; ++b)
        bo[b] = *(const bf16x8 *)(W + (size_t)(col0 + b * 32 + (lane & 31)) * K + kk);
    };
    auto step = [&](int k0, const bf16x8(&bo)[2]) {
      const int kk = k0 + (lane >> 5) * 8;
      bf16x8 ao[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) ao[a] = *(const bf16x8 *)&sH[a * 32 + (lane & 31)][kk];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bo[b], ao[a], acc[a][b], 0, 0, 0);
    };
    bf16x8 w0[2], w1[2], w2[2], w3[2];
    load_w(0, w0);
    load_w(16, w1);
    load_w(32, w2);
    load_w(48, w3);
#pragma unroll 1
    for (int k0 = 0; k0 < K; k0 += 64) {
      const bool more = k0 + 64 < K;
      step(k0, w0);
      if (more) load_w(k0 + 64, w0);
      step(k0 + 16, w1);
      if (more) load_w(k0 + 80, w1);
      step(k0 + 32, w2);
      if (more) load_w(k0 + 96, w2);
      step(k0 + 48, w3);
      if (more) load_w(k0 + 112, w3);
    }
    __syncthreads();  // every wave is done reading this layer's input
    const float *bias = bias_src + boff[l];
    // accumulator j of tile (a, b): feature col0 + 32 b + 8 (j / 4) + 4 (lane / 32) + j % 4
    // of row 32 a + lane % 32
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int row = a * 32 + (lane & 31);
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const int col = col0 + b * 32 + g * 8 + (lane >> 5) * 4;
          const float4 bc = *(const float4 *)(bias + col);
          const float v0 = acc[a][b][4 * g] + bc.x, v1 = acc[a][b][4 * g + 1] + bc.y,
                      v2 = acc[a][b][4 * g + 2] + bc.z, v3 = acc[a][b][4 * g + 3] + bc.w;
          if (l < 3) {
            const uint2 h = make_uint2(pack_bf16x2(gelu_f(v0), gelu_f(v1)),
                                       pack_bf16x2(gelu_f(v2), gelu_f(v3)));
            *(uint2 *)&sH[row][col] = h;
          } else {
            *(float4 *)&y[(row0 + row) * 256 + col] = make_float4(v0, v1, v2, v3);
          }
        }
      }
    __syncthreads();
  }
}

hipError_t mlp_infer(const uint16_t *x, int M, const uint16_t *wb, const float *bias_src, float *y,
                     hipStream_t st) {
  if (M % kInfRows) return hipErrorInvalidValue;
  hipLaunchKernelGGL(mlp_infer_kernel, dim3(M / kInfRows), dim3(256), 0, st, x, wb, bias_src, y);
  return hipGetLastError();
}

// ---------------------------------------------------------------- small kernels
__global__ void f32_to_bf16_kernel(const float *x, uint16_t *y, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = f2bf(x[i]);
}

// dZ_out = bf16(2 (Y - T) / (M N)); loss partial sums per block (deterministic
// second pass sums the blocks in order).
__global__ void mse_grad_kernel(const float *Y, const uint16_t *T, int64_t n, float scale,
                                uint16_t *dZ, float *block_loss) {
  __shared__ float red[256];
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float l = 0.0f;
  if (i < n) {
    const float d = Y[i] - bf2f(T[i]);
    dZ[i] = f2bf(2.0f * d * scale);
    l = d * d;
  }
  red[threadIdx.x] = l;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) block_loss[blockIdx.x] = red[0];
}

// One block: strided per-thread sums, then a tree (fixed order).
__global__ void sum_blocks_kernel(const float *part, int n, float scale, float *out) {
  __shared__ float red[256];
  float s = 0.0f;
  for (int i = threadIdx.x; i < n; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0] * scale;
}

// Column sums of a BF16 [M][N] matrix over a chunk of 64 rows per block
// (bias gradients); the chunks are then summed in order.
__global__ void colsum_bf16_kernel(const uint16_t *dZ, int M, int N, float *part) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int r0 = blockIdx.y * 64;
  if (c >= N) return;
  float s = 0.0f;
  for (int r = r0; r < r0 + 64 && r < M; ++r) s += bf2f(dZ[(size_t)r * N + c]);
  part[(size_t)blockIdx.y * N + c] = s;
}

// Sum of split-K partial products, fixed order.
__global__ void reduce_splits_kernel(const float *part, int splits, int64_t n, float *out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.0f;
  for (int k = 0; k < splits; ++k) s += part[(size_t)k * n + i];
  out[i] = s;
}

// Adam on FP32 master weights; refreshes the BF16 copy.
__global__ void adam_kernel(float *w, float *m, float *v, const float *g, uint16_t *wb,
                            int64_t n, float lr, float b1, float b2, float eps, float c1,
                            float c2) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / c1, vh = vi / c2;
  const float wi = w[i] - lr * mh / (sqrtf(vh) + eps);
  w[i] = wi;
  wb[i] = f2bf(wi);
}

hipError_t launch_f32_to_bf16(const float *x, uint16_t *y, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(f32_to_bf16_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                     x, y, n);
  return hipGetLastError();
}

hipError_t launch_mse_grad(const float *Y, const uint16_t *T, int64_t n, float scale,
                           uint16_t *dZ, float *block_loss, float *loss_out, hipStream_t st) {
  const unsigned nb = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(mse_grad_kernel, dim3(nb), dim3(256), 0, st, Y, T, n, scale, dZ,
                     block_loss);
  hipLaunchKernelGGL(sum_blocks_kernel, dim3(1), dim3(256), 0, st, block_loss, (int)nb, scale,
                     loss_out);
  return hipGetLastError();
}

hipError_t launch_colsum(const uint16_t *dZ, int M, int N, float *part, float *out,
                         hipStream_t st) {
  const int chunks = (M + 63) / 64;
  hipLaunchKernelGGL(colsum_bf16_kernel, dim3((N + 255) / 256, chunks), dim3(256), 0, st, dZ, M,
                     N, part);
  hipLaunchKernelGGL(reduce_splits_kernel, dim3((N + 255) / 256), dim3(256), 0, st, part,
                     chunks, (int64_t)N, out);
  return hipGetLastError();
}

hipError_t launch_reduce_splits(const float *part, int splits, int64_t n, float *out,
                                hipStream_t st) {
  hipLaunchKernelGGL(reduce_splits_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                     part, splits, n, out);
  return hipGetLastError();
}

hipError_t launch_adam(float *w, float *m, float *v, const float *g, uint16_t *wb, int64_t n,
                       float lr, float b1, float b2, float eps, float c1, float c2,
                       hipStream_t st) {
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, w, m, v,
                     g, wb, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace dock
