// Host side of the learned-proposal MLP: parameters, training step
// (forward, MSE loss, backward, Adam) and inference, all on the GPU.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "dock.h"
#include "mlp_internal.h"

using namespace dock;

namespace dock {
int abi_fail(int code, const char *fmt, ...);  // dock_abi.hip (thread-local last error)
int abi_check_device(const void *p, const char *what);  // dock_abi.hip
}

struct dock_mlp {
  int device = 0;
  int64_t step = 0;  // Adam steps taken
  float *w = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;  // FP32 [kMlpParams]
  uint16_t *wb = nullptr;                                         // BF16 copy
  // activations for up to `rows` rows
  int rows = 0;
  float *z1 = nullptr, *z2 = nullptr, *z3 = nullptr;
  uint16_t *a1 = nullptr, *a2 = nullptr, *a3 = nullptr, *dz0 = nullptr, *dz1 = nullptr;
  float *part = nullptr;  // split-K partial gradients [kMaxGradSplits][kMlpParams]
  float *block_loss = nullptr, *loss = nullptr;
  float *h_loss = nullptr;  // pinned
  std::mutex mu;
};

namespace {

constexpr int kMaxGradSplits = 64;

hipError_t alloc(void **p, size_t bytes) { return hipMalloc(p, bytes < 256 ? 256 : bytes); }

void free_rows(dock_mlp *n) {
  for (void *p : {(void *)n->z1, (void *)n->z2, (void *)n->z3, (void *)n->a1,
                  (void *)n->a2, (void *)n->a3, (void *)n->dz0, (void *)n->dz1,
                  (void *)n->part, (void *)n->block_loss})
    if (p) (void)hipFree(p);
  n->z1 = n->z2 = n->z3 = nullptr;
  n->a1 = n->a2 = n->a3 = n->dz0 = n->dz1 = nullptr;
  n->part = n->block_loss = nullptr;
  n->rows = 0;
}

int ensure_rows(dock_mlp *n, int M) {
  if (M <= n->rows) return DOCK_OK;
  free_rows(n);
  const size_t f = sizeof(float) * (size_t)M * 256, h = sizeof(uint16_t) * (size_t)M * 256;
  hipError_t e = hipSuccess;
  auto A = [&](void **p, size_t b) {
    if (e == hipSuccess) e = alloc(p, b);
  };
  A((void **)&n->z1, f);
  A((void **)&n->z2, f);
  A((void **)&n->z3, f);
  A((void **)&n->a1, h);
  A((void **)&n->a2, h);
  A((void **)&n->a3, h);
  A((void **)&n->dz0, h);
  A((void **)&n->dz1, h);
  A((void **)&n->part, sizeof(float) * kMaxGradSplits * kMlpParams);
  A((void **)&n->block_loss, sizeof(float) * ((size_t)M / 16 + 1));
  if (e != hipSuccess) {
    free_rows(n);
    return abi_fail(DOCK_E_NOMEM, "MLP activation buffers for %d rows: %s", M,
                    hipGetErrorString(e));
  }
  n->rows = M;
  return DOCK_OK;
}

// Split-K count of the weight gradients of M rows: about 256 rows per split
// (one staged panel), the rows of a split a multiple of 16, at most 64.
int grad_splits(int M) {
  const int s0 = min(kMaxGradSplits, (M + 255) / 256);
  for (int s = s0; s <= kMaxGradSplits; ++s)
    if (M % (16 * s) == 0) return s;
  for (int s = s0; s > 1; --s)
    if (M % (16 * s) == 0) return s;
  return 1;
}

// Training forward pass of M rows: layers 1-3 keep pre-activations (FP32)
// and activations (BF16); layer 4's epilogue turns its output straight into
// the MSE gradient dz0 and per-tile squared errors (the output itself is not
// stored).
hipError_t train_forward(dock_mlp *n, const uint16_t *x, const uint16_t *t, int M,
                         hipStream_t st) {
  const uint16_t *in[4] = {x, n->a1, n->a2, n->a3};
  const int kin[4] = {64, 256, 256, 256};
  const int64_t woff[4] = {kMlpW1, kMlpW2, kMlpW3, kMlpW4};
  const int64_t boff[4] = {kMlpB1, kMlpB2, kMlpB3, kMlpB4};
  float *zs[3] = {n->z1, n->z2, n->z3};
  uint16_t *as[3] = {n->a1, n->a2, n->a3};
  for (int l = 0; l < 4; ++l) {
    GemmArgs g{};
    g.A = in[l];
    g.lda = kin[l];
    g.B = n->wb + woff[l];  // storage [out][in]
    g.ldb = kin[l];
    g.ldc = 256;
    g.k_per_split = kin[l];
    g.bias = n->w + boff[l];
    if (l < 3) {
      g.Cf = zs[l];
      g.Cb = as[l];
    } else {
      g.Cb = n->dz0;
      g.target = t;
      g.scale = 1.0f / ((float)M * 256.0f);
      g.block_loss = n->block_loss;
    }
    hipError_t e = gemm_bf16(g, false, true, l < 3 ? kEpiBiasGelu : kEpiBiasMse, M, 256, 1, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

extern "C" {

size_t dock_mlp_param_count(void) { return (size_t)kMlpParams; }

int dock_mlp_create(const float *init_params, dock_mlp **out) {
  if (!out) return abi_fail(DOCK_E_INVAL, "out is NULL");
  *out = nullptr;
  if (!init_params) return abi_fail(DOCK_E_INVAL, "init_params is NULL");
  dock_mlp *n = new (std::nothrow) dock_mlp;
  if (!n) return abi_fail(DOCK_E_NOMEM, "host allocation");
  const size_t pb = sizeof(float) * kMlpParams;
  hipError_t e = hipGetDevice(&n->device);
  auto A = [&](void **p, size_t b) {
    if (e == hipSuccess) e = alloc(p, b);
  };
  A((void **)&n->w, pb);
  A((void **)&n->m, pb);
  A((void **)&n->v, pb);
  A((void **)&n->g, pb);
  A((void **)&n->wb, sizeof(uint16_t) * kMlpParams);
  A((void **)&n->loss, sizeof(float));
  if (e == hipSuccess) e = hipHostMalloc((void **)&n->h_loss, sizeof(float), 0);
  if (e == hipSuccess) e = hipMemcpy(n->w, init_params, pb, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(n->m, 0, pb);
  if (e == hipSuccess) e = hipMemset(n->v, 0, pb);
  if (e == hipSuccess) e = launch_f32_to_bf16(n->w, n->wb, kMlpParams, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    int rc = abi_fail(DOCK_E_DEVICE, "dock_mlp_create: %s", hipGetErrorString(e));
    dock_mlp_free(n);
    return rc;
  }
  *out = n;
  return DOCK_OK;
}

void dock_mlp_free(dock_mlp *n) {
  if (!n) return;
  (void)hipDeviceSynchronize();
  free_rows(n);
  for (void *p : {(void *)n->w, (void *)n->m, (void *)n->v, (void *)n->g, (void *)n->wb,
                  (void *)n->loss})
    if (p) (void)hipFree(p);
  if (n->h_loss) (void)hipHostFree(n->h_loss);
  delete n;
}

int dock_mlp_get_params(dock_mlp *n, float *host_params) {
  if (!n || !host_params) return abi_fail(DOCK_E_INVAL, "NULL argument");
  hipError_t e = hipMemcpy(host_params, n->w, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost);
  return e == hipSuccess ? DOCK_OK : abi_fail(DOCK_E_DEVICE, "%s", hipGetErrorString(e));
}

int dock_mlp_set_params(dock_mlp *n, const float *host_params) {
  if (!n || !host_params) return abi_fail(DOCK_E_INVAL, "NULL argument");
  hipError_t e = hipMemcpy(n->w, host_params, sizeof(float) * kMlpParams, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = launch_f32_to_bf16(n->w, n->wb, kMlpParams, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  return e == hipSuccess ? DOCK_OK : abi_fail(DOCK_E_DEVICE, "%s", hipGetErrorString(e));
}

int dock_mlp_forward(dock_mlp *n, const uint16_t *x_bf16, int M, float *y, void *stream) {
  if (!n || !x_bf16 || !y) return abi_fail(DOCK_E_INVAL, "NULL argument");
  if (M < 64 || M % 64) return abi_fail(DOCK_E_INVAL, "rows must be a positive multiple of 64");
  int rc = abi_check_device(x_bf16, "x");
  if (rc == DOCK_OK) rc = abi_check_device(y, "y");
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(n->mu);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = mlp_infer(x_bf16, M, n->wb, n->w, y, st);
  return e == hipSuccess ? DOCK_OK : abi_fail(DOCK_E_DEVICE, "mlp forward: %s", hipGetErrorString(e));
}

int dock_mlp_loss_grad(dock_mlp *n, const uint16_t *x_bf16, const uint16_t *t_bf16, int M,
                       float *grad_out, float *loss_out, void *stream) {
  if (!n || !x_bf16 || !t_bf16) return abi_fail(DOCK_E_INVAL, "NULL argument");
  if (M < 64 || M % 64) return abi_fail(DOCK_E_INVAL, "rows must be a positive multiple of 64");
  int rc = abi_check_device(x_bf16, "x");
  if (rc == DOCK_OK) rc = abi_check_device(t_bf16, "t");
  if (rc == DOCK_OK) rc = abi_check_device(grad_out, "grad_out");
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(n->mu);
  rc = ensure_rows(n, M);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = train_forward(n, x_bf16, t_bf16, M, st);
  if (e == hipSuccess && loss_out)
    e = launch_sum_blocks(n->block_loss, M / 16, 1.0f / ((float)M * 256.0f), n->loss, st);
  // backward, layer 4 .. 1: the weight and bias gradients of a layer (split
  // over the rows; the splits summed once at the end), then dZ of the layer
  // below through the GELU derivative
  const int splits = grad_splits(M);
  const uint16_t *acts[4] = {x_bf16, n->a1, n->a2, n->a3};
  const float *pre[4] = {nullptr, n->z1, n->z2, n->z3};
  const int kin[4] = {64, 256, 256, 256};
  const int64_t woff[4] = {kMlpW1, kMlpW2, kMlpW3, kMlpW4};
  uint16_t *dz = n->dz0, *dz_next = n->dz1;
  for (int l = 3; l >= 0 && e == hipSuccess; --l) {
    GemmArgs w{};
    w.A = dz;  // storage [M][256] read as [k = row][m = out]
    w.lda = 256;
    w.B = acts[l];  // storage [M][in] read as [k = row][n = in]
    w.ldb = kin[l];
    w.ldc = kin[l];
    w.k_per_split = M / splits;
    w.split_stride = kMlpParams;
    w.Cf = (splits > 1 ? n->part : n->g) + woff[l];
    GemmArgs g{};
    if (l > 0) {
      g.A = dz;  // [M][256]
      g.lda = 256;
      g.B = n->wb + woff[l];  // W_l storage [out=256][in] = [k][n]
      g.ldb = kin[l];
      g.ldc = kin[l];
      g.k_per_split = 256;
      g.Cb = dz_next;
      g.aux = pre[l];
    }
    e = backward_layer(w, kin[l], splits, l > 0 ? &g : nullptr, M, st);
    uint16_t *t = dz;
    dz = dz_next;
    dz_next = t;
  }
  if (e == hipSuccess && splits > 1) e = launch_reduce_grads(n->part, splits, kMlpParams, n->g, st);
  if (e == hipSuccess && grad_out)
    e = hipMemcpyAsync(grad_out, n->g, sizeof(float) * kMlpParams, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess && loss_out) {
    e = hipMemcpyAsync(n->h_loss, n->loss, sizeof(float), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess) *loss_out = *(volatile float *)n->h_loss;
  }
  return e == hipSuccess ? DOCK_OK : abi_fail(DOCK_E_DEVICE, "mlp backward: %s", hipGetErrorString(e));
}

int dock_mlp_adam(dock_mlp *n, float lr, float beta1, float beta2, float eps, void *stream) {
  if (!n) return abi_fail(DOCK_E_INVAL, "NULL argument");
  if (!(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
      !(eps > 0.0f))
    return abi_fail(DOCK_E_INVAL, "bad Adam hyper-parameters");
  std::lock_guard<std::mutex> lk(n->mu);
  n->step += 1;
  const float c1 = (float)(1.0 - std::pow((double)beta1, (double)n->step));
  const float c2 = (float)(1.0 - std::pow((double)beta2, (double)n->step));
  hipError_t e = launch_adam(n->w, n->m, n->v, n->g, n->wb, kMlpParams, lr, beta1, beta2, eps, c1,
                             c2, (hipStream_t)stream);
  return e == hipSuccess ? DOCK_OK : abi_fail(DOCK_E_DEVICE, "adam: %s", hipGetErrorString(e));
}

}  // extern "C"

namespace dock {
void mlp_export_weights(dock_mlp *n, const uint16_t **wb, const float **w) {
  *wb = n->wb;
  *w = n->w;
}
}  // namespace dock
