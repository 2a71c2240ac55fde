// Benchmark probes (instrumentation, not part of the docking path).
//
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

// VALU issue probe: kProbeChains independent dependency chains per lane, so
// the issue rate, not latency, bounds the kernel.  kind 0: one FP32 FMA per
// chain and iteration; kind 1: the sweep's per-evaluation mix (6 FMAs placing
// a point in voxel units, the voxel offset -- 3 clamps, 3 conversions, 2
// 24-bit multiply-adds, as voxel_byte_offset does it -- then a conversion and
// an add folding the offset back into the chain): 16 VALU instructions.
// The multiplier and addend come from the arguments, so nothing is folded at
// compile time.
constexpr int kProbeChains = 8;

__global__ void __launch_bounds__(kProbeThreads)
    valu_probe_kernel(int kind, int iters, float a, float b, GridScaled gs, float *out) {
  const uint32_t tid = blockIdx.x * kProbeThreads + threadIdx.x;
  float acc[kProbeChains];
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) acc[c] = (float)(c + (tid & 7));
  if (kind == 0) {
    for (int i = 0; i < iters; ++i) {
#pragma unroll
      for (int c = 0; c < kProbeChains; ++c) acc[c] = fmaf(acc[c], a, b);
    }
  } else {
    for (int i = 0; i < iters; ++i) {
#pragma unroll
      for (int c = 0; c < kProbeChains; ++c) {
        const float p = acc[c];
        const float tx = fmaf(b, a, fmaf(a, b, p));
        const float ty = fmaf(b, p, fmaf(a, p, b));
        const float tz = fmaf(p, b, fmaf(p, a, a));
        const uint32_t off = voxel_byte_offset(gs, tx, ty, tz);
        acc[c] = p + (float)off;
      }
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) s += acc[c];
  out[tid] = s;
}

}  // namespace
}  // namespace dock

extern "C" int dock_probe_valu(int kind, int blocks, int iters, float *out, float *ms, void *stream) {
  using namespace dock;
  if (!out || !ms) return abi_fail(DOCK_E_INVAL, "NULL argument");
  if (kind != 0 && kind != 1) return abi_fail(DOCK_E_INVAL, "kind must be 0 or 1");
  if (blocks < 1 || blocks > (1 << 20)) return abi_fail(DOCK_E_LIMIT, "blocks outside [1, 2^20]");
  if (iters < 1 || iters > (1 << 20)) return abi_fail(DOCK_E_LIMIT, "iters outside [1, 2^20]");
  int rc = abi_check_device(out, "out");
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipError_t e = hipEventCreate(&ev[0]);
  if (e == hipSuccess) e = hipEventCreate(&ev[1]);
  if (e == hipSuccess) e = hipEventRecord(ev[0], st);
  if (e == hipSuccess) {
    // kind 0 adds 1 per FMA (a = b = 1); kind 1 keeps its points inside a
    // 64^3 box (a = 1/4, b = 1/8, zero offsets would fold nothing away)
    const float a = kind == 0 ? 1.0f : 0.25f, b = kind == 0 ? 1.0f : 0.125f;
    const GridScaled gs{63.5f, 63.5f, 63.5f, 64u, 256u};
    hipLaunchKernelGGL(valu_probe_kernel, dim3((unsigned)blocks), dim3(kProbeThreads), 0, st, kind,
                       iters, a, b, gs, out);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(ev[1], st);
  if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, ev[0], ev[1]);
  for (hipEvent_t x : ev)
    if (x) (void)hipEventDestroy(x);
  return e == hipSuccess ? DOCK_OK : abi_fail(DOCK_E_DEVICE, "VALU probe: %s", hipGetErrorString(e));
}

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
