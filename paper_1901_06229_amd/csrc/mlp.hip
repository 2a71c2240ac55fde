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

constexpr int kTile = 64;   // output tile edge
constexpr int kKc = 256;    // K staged in LDS at once (the whole K of every product but the
                            // weight gradients of large batches)
// A staged panel row holds k in 16-byte chunks of 8; chunk j of row r is
// stored at chunk j ^ ((r / 8) mod 8), so the rows 8 apart that one wave
// writes in a transposing stage (and the 32 rows an operand read spans) fall
// on different LDS banks, while each 8-value operand stays contiguous.
__device__ __forceinline__ int swz(int r, int k) { return (((k >> 3) ^ ((r >> 3) & 7)) << 3) | (k & 7); }

// A 64 x kc panel ([row][k], k contiguous) staged into LDS in two steps, so
// that both operands' loads are in flight before either is written: every
// thread loads up to 8 16-byte chunks, then writes them.  T: the source is
// stored [k][row] (64 contiguous rows per k), else [row][k] with kc a power
// of two.  Loads are unconditional (a thread past the panel re-reads its
// last chunk); only the LDS writes are predicated.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
struct Panel {
  u32x4 v[8];
};

template <bool T>
__device__ __forceinline__ void load_panel(Panel &p, const uint16_t *src, int ld, int r0, int k0,
                                           int kc, int tid) {
  const int nch = 8 * kc;
  const int lg = __builtin_ctz((unsigned)kc) - 3, per = 1 << lg;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int e = min(tid + 256 * i, nch - 1);
    if (!T) {
      const int r = e >> lg, c = (e & (per - 1)) * 8;
      p.v[i] = *(const u32x4 *)(src + (size_t)(r0 + r) * ld + k0 + c);
    } else {
      const int kr = e >> 3, c = (e & 7) * 8;
      p.v[i] = *(const u32x4 *)(src + (size_t)(k0 + kr) * ld + r0 + c);
    }
  }
}

template <bool T>
__device__ __forceinline__ void store_panel(const Panel &p, uint16_t (*s)[kKc], int kc,
                                            int tid) {
  const int nch = 8 * kc;
  const int lg = __builtin_ctz((unsigned)kc) - 3, per = 1 << lg;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int e = tid + 256 * i;
    if (e < nch) {
      if (!T) {
        const int r = e >> lg, c = (e & (per - 1)) * 8;
        *(u32x4 *)&s[r][swz(r, c)] = p.v[i];
      } else {
        const int kr = e >> 3, c = (e & 7) * 8;
        const uint16_t *h = (const uint16_t *)&p.v[i];
#pragma unroll
        for (int q = 0; q < 8; ++q) s[c + q][swz(c + q, kr)] = h[q];
      }
    }
  }
}

// C[m][n] = sum_k opA[m][k] * opB[k][n]
//   opA[m][k] = TA ? A[k * lda + m] : A[m * lda + k]
//   opB[k][n] = TB ? B[n * ldb + k] : B[k * ldb + n]
// One 64 x 64 output tile (column tile bx, row tile by) over the K range
// of split bz, staged 256 at a time; M, N multiples of 64, the K of a split
// a multiple of 16.  tile_id numbers the tile for the per-tile loss.
struct GemmLds {
  uint16_t sA[kTile][kKc];  // [m][k], swizzled
  uint16_t sB[kTile][kKc];  // [n][k], swizzled
  float sRed[256];
};

template <bool TA, bool TB, int EPI>
__device__ __forceinline__ void gemm_tile(const GemmArgs &g, GemmLds &L, int bx, int by, int bz,
                                          int tile_id) {
  auto &sA = L.sA;
  auto &sB = L.sB;
  float *sRed = L.sRed;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int m0 = by * kTile, n0 = bx * kTile;
  const int split = bz;
  const int kb = g.k_per_split * split, ke = kb + g.k_per_split;
  const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;
  // weight gradients: the first column of blocks also sums its rows of opA
  // (the bias gradient), thread t over k = t mod 4 of row t / 4
  const bool bias_sum = EPI == kEpiWgrad && bx == 0;
  f32x16 acc;
#pragma unroll
  for (int j = 0; j < 16; ++j) acc[j] = 0.0f;
  float bsum = 0.0f;

  for (int k0 = kb; k0 < ke; k0 += kKc) {
    const int kc = min(kKc, ke - k0);
    {
      Panel pa, pb;
      load_panel<TA>(pa, g.A, g.lda, m0, k0, kc, tid);
      load_panel<!TB>(pb, g.B, g.ldb, n0, k0, kc, tid);
      // keep the loads here (not sunk next to their predicated writes), so
      // all of them are in flight together
#pragma unroll
      for (int i = 0; i < 8; ++i) asm volatile("" ::"v"(pa.v[i]), "v"(pb.v[i]));
      store_panel<TA>(pa, sA, kc, tid);
      store_panel<!TB>(pb, sB, kc, tid);
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < kc; kk += 16) {
      const int koff = kk + (lane >> 5) * 8;
      const int ra = wm + (lane & 31), rb = wn + (lane & 31);
      const bf16x8 a = *(const bf16x8 *)&sA[ra][swz(ra, koff)];
      const bf16x8 b = *(const bf16x8 *)&sB[rb][swz(rb, koff)];
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    if (bias_sum)
      for (int k = tid & 3; k < kc; k += 4) bsum += bf2f(sA[tid >> 2][swz(tid >> 2, k)]);
    __syncthreads();
  }

  float *dst = g.Cf + (EPI == kEpiWgrad ? (size_t)split * g.split_stride : 0);
  if (bias_sum) {
    // bias gradient (stored after the weight matrix): the four partial sums
    // of a row added in order
    sRed[tid] = bsum;
    __syncthreads();
    if (tid < kTile) {
      const float *q = sRed + 4 * tid;
      dst[(size_t)256 * g.ldc + m0 + tid] = ((q[0] + q[1]) + q[2]) + q[3];
    }
  }
  const int col = n0 + wn + (lane & 31);
  float l2 = 0.0f;
  // operands of the epilogue loaded up front (the targets share their type
  // with the BF16 output, so the compiler would not move their loads ahead
  // of the stores)
  float ep[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int row = m0 + wm + (j >> 2) * 8 + (lane >> 5) * 4 + (j & 3);
    const size_t at = (size_t)row * g.ldc + col;
    if (EPI == kEpiBiasMse) ep[j] = bf2f(g.target[at]);
    if (EPI == kEpiGeluGrad) ep[j] = g.aux[at];
  }
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int row = m0 + wm + (j >> 2) * 8 + (lane >> 5) * 4 + (j & 3);
    const size_t at = (size_t)row * g.ldc + col;
    float v = acc[j];
    if (EPI == kEpiWgrad) {
      dst[at] = v;
    } else if (EPI == kEpiBiasGelu) {
      v += g.bias[col];
      g.Cf[at] = v;                    // pre-activation, kept for the backward pass
      g.Cb[at] = f2bf(gelu_f(v));      // activation, BF16
    } else if (EPI == kEpiBiasMse) {   // dZ = bf16(2 (Y - T) scale), Y = output + bias
      const float d = (v + g.bias[col]) - ep[j];
      g.Cb[at] = f2bf(2.0f * d * g.scale);
      l2 += d * d;
    } else if (EPI == kEpiGeluGrad) {  // dZ_prev = bf16(dA * gelu'(Z_prev))
      g.Cb[at] = f2bf(v * gelu_grad_f(ep[j]));
    }
  }
  if (EPI == kEpiBiasMse) {
    // squared error of the tile: fixed-order tree over the block
    sRed[tid] = l2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (tid < w) sRed[tid] += sRed[tid + w];
      __syncthreads();
    }
    if (tid == 0) g.block_loss[tile_id] = sRed[0];
  }
}

template <bool TA, bool TB, int EPI>
__global__ void __launch_bounds__(256) gemm_bf16_kernel(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) GemmLds L;
  gemm_tile<TA, TB, EPI>(g, L, blockIdx.x, blockIdx.y, blockIdx.z,
                         blockIdx.y * gridDim.x + blockIdx.x);
}

// One backward step of a layer in one launch: the first w_tiles blocks are
// the weight / bias gradient tiles (w: wx column tiles x 4 row tiles x
// splits), the rest the tiles of dZ of the layer below (d: dx column tiles
// per 64 rows).  Both read the layer's dZ only.
__global__ void __launch_bounds__(256) backward_kernel(GemmArgs w, GemmArgs d, int wx, int splits,
                                                       int dx) {
  __shared__ __attribute__((aligned(16))) GemmLds L;
  const int b = blockIdx.x, w_tiles = wx * 4 * splits;
  if (b < w_tiles) {
    const int bz = b / (wx * 4), r = b - bz * wx * 4;
    gemm_tile<true, false, kEpiWgrad>(w, L, r % wx, r / wx, bz, 0);
  } else {
    const int t = b - w_tiles;
    gemm_tile<false, false, kEpiGeluGrad>(d, L, t % dx, t / dx, 0, 0);
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
  if (M % kTile || N % kTile || g.k_per_split % 16 || g.k_per_split < 16 || splits < 1)
    return hipErrorInvalidValue;
  // a panel stored [row][k] is staged with shifts: its K chunks are powers of two
  if ((!ta || tb) && (g.k_per_split & (g.k_per_split - 1))) return hipErrorInvalidValue;
#define DOCK_GEMM(TA, TB, E) \
  if (ta == TA && tb == TB && epi == E) return gemm_t<TA, TB, E>(g, M, N, splits, st);
  DOCK_GEMM(false, true, kEpiBiasGelu)
  DOCK_GEMM(false, true, kEpiBiasMse)
#undef DOCK_GEMM
  return hipErrorInvalidValue;
}

hipError_t backward_layer(const GemmArgs &w, int in, int splits, const GemmArgs *d, int M,
                          hipStream_t st) {
  // d stages its dZ panel [row][k] with shifts: a power-of-two K
  if (in % kTile || w.k_per_split % 16 || w.k_per_split < 16 || splits < 1 ||
      (d && (M % kTile || d->k_per_split % 16 || d->k_per_split < 16 ||
             (d->k_per_split & (d->k_per_split - 1)))))
    return hipErrorInvalidValue;
  const int wx = in / kTile, dx = in / kTile;
  const int blocks = wx * 4 * splits + (d ? dx * (M / kTile) : 0);
  hipLaunchKernelGGL(backward_kernel, dim3((unsigned)blocks), dim3(256), 0, st, w,
                     d ? *d : GemmArgs{}, wx, splits, dx);
  return hipGetLastError();
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

// Gradient = sum of the split-K partial gradients (each a whole parameter
// vector), in split order.
__global__ void reduce_grads_kernel(const float *part, int splits, int64_t n, float *out) {
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

hipError_t launch_sum_blocks(const float *block_loss, int n, float scale, float *loss_out,
                             hipStream_t st) {
  hipLaunchKernelGGL(sum_blocks_kernel, dim3(1), dim3(256), 0, st, block_loss, n, scale,
                     loss_out);
  return hipGetLastError();
}

hipError_t launch_reduce_grads(const float *part, int splits, int64_t n, float *out,
                               hipStream_t st) {
  hipLaunchKernelGGL(reduce_grads_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
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
