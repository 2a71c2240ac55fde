// Random-gather probe: the sustained rate of scattered 4-byte reads from a
// buffer of a given size, the denominator for the voxel gathers of the sweep
// and alignment kernels.  Every lane draws its own addresses (xorshift32),
// so a wave's 64 reads touch 64 unrelated cache lines; a buffer that fits the
// L2 measures L2 lines, a larger one the Infinity Cache / HBM path.
#include <hip/hip_runtime.h>

#include "dock.h"
#include "sweep_common.h"

namespace dock {
int abi_fail(int code, const char *fmt, ...);  // dock_abi.hip (thread-local last error)
int abi_check_device(const void *p, const char *what);

namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeUnroll = 8;

__global__ void __launch_bounds__(kProbeThreads)
    gather_probe_kernel(const float *buf, uint32_t n_floats, uint32_t mask, int iters, float *out) {
  const uint32_t tid = blockIdx.x * kProbeThreads + threadIdx.x;
  const __amdgpu_buffer_rsrc_t r =
      __builtin_amdgcn_make_buffer_rsrc((void *)buf, (short)0, (int)(4u * n_floats), 0x00020000);
  uint32_t x = 0x9E3779B9u ^ (tid * 2654435761u + 1u);
  float s = 0.0f;
  for (int i = 0; i < iters; i += kProbeUnroll) {
    float v[kProbeUnroll];
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) {
      x ^= x << 13;
      x ^= x >> 17;
      x ^= x << 5;
      v[u] = grid_load(r, (x & mask) << 2);
    }
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) s += v[u];
  }
  out[tid] = s;
}

}  // namespace
}  // namespace dock

extern "C" int dock_probe_gather(const float *buf, int log2_floats, int blocks, int iters, float *out,
                                 float *ms, void *stream) {
  using namespace dock;
  if (!buf || !out || !ms) return abi_fail(DOCK_E_INVAL, "NULL argument");
  if (log2_floats < 6 || log2_floats > 28) return abi_fail(DOCK_E_LIMIT, "log2_floats outside [6, 28]");
  if (blocks < 1 || blocks > (1 << 20)) return abi_fail(DOCK_E_LIMIT, "blocks outside [1, 2^20]");
  if (iters < kProbeUnroll || iters > (1 << 16) || iters % kProbeUnroll)
    return abi_fail(DOCK_E_LIMIT, "iters must be a multiple of 8 in [8, 65536]");
  int rc = abi_check_device(buf, "buf");
  if (rc == DOCK_OK) rc = abi_check_device(out, "out");
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipError_t e = hipEventCreate(&ev[0]);
  if (e == hipSuccess) e = hipEventCreate(&ev[1]);
  if (e == hipSuccess) e = hipEventRecord(ev[0], st);
  if (e == hipSuccess) {
    const uint32_t n = 1u << log2_floats;
    hipLaunchKernelGGL(gather_probe_kernel, dim3((unsigned)blocks), dim3(kProbeThreads), 0, st, buf, n,
                       n - 1u, iters, out);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(ev[1], st);
  if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, ev[0], ev[1]);
  for (hipEvent_t x : ev)
    if (x) (void)hipEventDestroy(x);
  return e == hipSuccess ? DOCK_OK : abi_fail(DOCK_E_DEVICE, "gather probe: %s", hipGetErrorString(e));
}
