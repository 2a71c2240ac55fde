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

enum GemmEpilogue { kEpiWgrad = 0, kEpiBiasGelu = 1, kEpiBiasMse = 2, kEpiGeluGrad = 3 };

struct GemmArgs {
  const uint16_t *A;  // BF16
  const uint16_t *B;  // BF16
  int lda, ldb, ldc;
  int k_per_split;
  int64_t split_stride;  // elements between split-K partial outputs (kEpiWgrad)
  float *Cf;             // FP32 output (pre-activation / weight gradient, then bias gradient)
  uint16_t *Cb;          // BF16 output (activation / gradient)
  const float *bias;
  const float *aux;      // pre-activation for the GELU derivative
  const uint16_t *target;  // kEpiBiasMse: BF16 targets, same layout as the output
  float scale;             // kEpiBiasMse: 1 / (rows x outputs)
  float *block_loss;       // kEpiBiasMse: squared error per output tile
};

// Epilogues: kEpiBiasGelu (Cf = pre-activation, Cb = GELU), kEpiBiasMse
// (Cb = MSE gradient of output + bias against target, per-tile squared
// error), kEpiGeluGrad (Cb = bf16(product x GELU'(aux))), kEpiWgrad (opA =
// dZ^T, opB = activations: Cf + split x split_stride = the split's weight
// gradient [M][ldc], then its bias gradient [M] = row sums of opA).
hipError_t gemm_bf16(const GemmArgs &g, bool ta, bool tb, int epi, int M, int N, int splits,
                     hipStream_t st);
// Backward step of a layer with `in` inputs in one launch: the weight and
// bias gradient (w: kEpiWgrad over the rows, `splits` splits) and, if d is
// not null, dZ of the layer below for M rows (d: kEpiGeluGrad).
hipError_t backward_layer(const GemmArgs &w, int in, int splits, const GemmArgs *d, int M,
                          hipStream_t st);
hipError_t launch_f32_to_bf16(const float *x, uint16_t *y, int64_t n, hipStream_t st);
hipError_t launch_sum_blocks(const float *block_loss, int n, float scale, float *loss_out,
                             hipStream_t st);
hipError_t launch_reduce_grads(const float *part, int splits, int64_t n, float *out,
                               hipStream_t st);
hipError_t launch_adam(float *w, float *m, float *v, const float *g, uint16_t *wb, int64_t n,
                       float lr, float b1, float b2, float eps, float c1, float c2,
                       hipStream_t st);

// Fused forward pass (all layers in one kernel, activations in LDS) of M
// rows, M a multiple of 64; y = [M][256] FP32.
hipError_t mlp_infer(const uint16_t *x, int M, const uint16_t *wb, const float *bias_src, float *y,
                     hipStream_t st);

}  // namespace dock

struct dock_mlp;
namespace dock {
// Device pointers to the BF16 weight copy and the FP32 master parameters.
void mlp_export_weights(dock_mlp *n, const uint16_t **wb, const float **w);
}  // namespace dock
