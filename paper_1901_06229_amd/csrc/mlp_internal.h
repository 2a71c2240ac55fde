// Internal interface of the MLP kernels (learned angle proposal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dock {

constexpr int kMlpIn = 64, kMlpHid = 256, kMlpOut = 256;
// packed FP32 parameters: W1[256][64] b1 W2[256][256] b2 W3 b3 W4 b4
constexpr int64_t kMlpW1 = 0, kMlpB1 = kMlpW1 + 256 * 64, kMlpW2 = kMlpB1 + 256,
                  kMlpB2 = kMlpW2 + 256 * 256, kMlpW3 = kMlpB2 + 256,
                  kMlpB3 = kMlpW3 + 256 * 256, kMlpW4 = kMlpB3 + 256,
                  kMlpB4 = kMlpW4 + 256 * 256, kMlpParams = kMlpB4 + 256;

enum GemmEpilogue { kEpiStore = 0, kEpiBiasGelu = 1, kEpiBias = 2, kEpiGeluGrad = 3 };

struct GemmArgs {
  const uint16_t *A;  // BF16
  const uint16_t *B;  // BF16
  int lda, ldb, ldc;
  int k_per_split;
  int64_t split_stride;  // elements between split-K partial outputs
  float *Cf;             // FP32 output (pre-activation / partials)
  uint16_t *Cb;          // BF16 output (activation / gradient)
  const float *bias;
  const float *aux;      // pre-activation for the GELU derivative
};

hipError_t gemm_bf16(const GemmArgs &g, bool ta, bool tb, int epi, int M, int N, int splits,
                     hipStream_t st);
hipError_t launch_f32_to_bf16(const float *x, uint16_t *y, int64_t n, hipStream_t st);
hipError_t launch_mse_grad(const float *Y, const uint16_t *T, int64_t n, float scale,
                           uint16_t *dZ, float *block_loss, float *loss_out, hipStream_t st);
hipError_t launch_colsum(const uint16_t *dZ, int M, int N, float *part, float *out,
                         hipStream_t st);
hipError_t launch_reduce_splits(const float *part, int splits, int64_t n, float *out,
                                hipStream_t st);
hipError_t launch_adam(float *w, float *m, float *v, const float *g, uint16_t *wb, int64_t n,
                       float lr, float b1, float b2, float eps, float c1, float c2,
                       hipStream_t st);

// Fused forward pass (all layers in one kernel, activations in LDS) of M
// rows, M a multiple of 64; y = [M][256] FP32.
hipError_t mlp_infer(const uint16_t *x, int M, const uint16_t *wb, const float *bias_src, float *y,
                     hipStream_t st);

// Forward pass of M rows (M a multiple of 64) with BF16 weights wb and FP32
// biases taken from the packed layout; z1..z3 / a1..a3 / y are caller
// buffers of M x 256.
hipError_t mlp_forward(const uint16_t *x, int M, const uint16_t *wb, const float *bias_src,
                       float *z1, uint16_t *a1, float *z2, uint16_t *a2, float *z3,
                       uint16_t *a3, float *y, hipStream_t st);

}  // namespace dock

struct dock_mlp;
namespace dock {
// Device pointers to the BF16 weight copy and the FP32 master parameters.
void mlp_export_weights(dock_mlp *n, const uint16_t **wb, const float **w);
}  // namespace dock
