// Rigid alignment search before the rotamer sweep (paper §3.1: the first
// phase treats the ligand as a rigid body and looks for the orientation that
// fits the pocket best, scoring every rotation; §4.1: rotation and scoring are
// fused so that no rotated pose is stored, a reduction picks the best
// orientation, and the ligand is rotated once).
//
// One wave per (ligand, orientation) item and one lane per candidate
// rotation.  The starting pose is staged in LDS as coordinates relative to
// its centroid, in voxel units; every lane reads the same atom at a time (an
// LDS broadcast), rotates it with its own matrix and accumulates the voxel
// values in atom order.  A wave reduction over (score, index) keys selects the
// best rotation, lowest index on ties.  The winner is not applied to a pose:
// it is folded into the item's rigid transform
//     X = R_a (R_o x + t_o - c) + c = (R_a R_o) x + (R_a (t_o - c) + c),
// which the sweep stages like any orientation.
#include "dock_internal.h"

namespace dock {
namespace {

constexpr int kAlignWaves = 4;
// items per launch: keeps the grid below 2^32 work-items per dimension
constexpr int64_t kAlignChunk = (int64_t)1 << 24;

template <int MAXN>
__global__ void __launch_bounds__(kAlignWaves * kWave) align_kernel(AlignArgs A, int64_t item0,
                                                                    int64_t n_items) {
  __shared__ float4 sZ[kAlignWaves][MAXN];
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  const int lane = threadIdx.x % kWave;
  const int64_t item = item0 + (int64_t)blockIdx.x * kAlignWaves + wv;
  if (item >= n_items) return;
  const int O = A.n_orient;
  const int l = (int)(item / O), o = (int)(item - (int64_t)l * O);
  if (A.status[l] != 0) {
    if (lane == 0) A.item_align[item] = -1;
    return;
  }
  const int a0 = A.lig.atom_offset[l];
  const int n = A.lig.atom_offset[l + 1] - a0;  // 1 .. MAXN once validated
  float4 *Z = sZ[wv];
  const float *T = A.orient + 12 * (size_t)o;

  // starting pose, and its centroid from fixed-order sums
  float sx = 0.0f, sy = 0.0f, sz = 0.0f;
  for (int i = lane; i < n; i += kWave) {
    const float *p = A.lig.xyz + 3 * (size_t)(a0 + i);
    const float3 x = orient_point(T, p[0], p[1], p[2]);
    Z[i] = make_float4(x.x, x.y, x.z, 0.0f);
    sx += x.x;
    sy += x.y;
    sz += x.z;
  }
  const float fn = (float)n;
  const float cx = wave_sum(sx) / fn, cy = wave_sum(sy) / fn, cz = wave_sum(sz) / fn;
  const GridView G = A.grid;
  const float ih = G.inv_h;
  // each lane rewrites the atoms it wrote, so only the read loop below needs the sync
  for (int i = lane; i < n; i += kWave) {
    const float4 x = Z[i];
    Z[i] = make_float4((x.x - cx) * ih, (x.y - cy) * ih, (x.z - cz) * ih, 0.0f);
  }
  wave_lds_sync();

  // centroid in voxel units: a rotated atom sits at q + R z
  const float qx = (cx - G.ox) * ih, qy = (cy - G.oy) * ih, qz = (cz - G.oz) * ih;
  const GridScaled GS = grid_scaled(G);
  const __amdgpu_buffer_rsrc_t grsrc = grid_rsrc(G);
  uint64_t best = 0;
  for (int c0 = 0; c0 < A.n_align; c0 += kWave) {
    const int a = c0 + lane;
    const float *Rm = A.rot + 9 * (size_t)min(a, A.n_align - 1);
    const float m0 = Rm[0], m1 = Rm[1], m2 = Rm[2], m3 = Rm[3], m4 = Rm[4], m5 = Rm[5],
                m6 = Rm[6], m7 = Rm[7], m8 = Rm[8];
    float s = 0.0f;
#pragma unroll 4
    for (int i = 0; i < n; ++i) {
      const float4 z = Z[i];
      const float tx = fmaf(m0, z.x, fmaf(m1, z.y, fmaf(m2, z.z, qx)));
      const float ty = fmaf(m3, z.x, fmaf(m4, z.y, fmaf(m5, z.z, qy)));
      const float tz = fmaf(m6, z.x, fmaf(m7, z.y, fmaf(m8, z.z, qz)));
      s += grid_load(grsrc, voxel_byte_offset(GS, tx, ty, tz));
    }
    if (a < A.n_align) {
      const uint64_t k = best_key(s, (uint32_t)a);
      best = k > best ? k : best;
    }
  }
  best = wave_max_u64(best);
  const int a = (int)key_index(best);

  // fold the winner into the item's transform: lanes 0-8 the matrix entries,
  // lanes 9-11 the translation
  const float *Ra = A.rot + 9 * (size_t)a;
  float v = 0.0f;
  if (lane < 9) {
    const int d = lane / 3, e = lane - 3 * d;
    v = fmaf(Ra[3 * d], T[e], fmaf(Ra[3 * d + 1], T[3 + e], Ra[3 * d + 2] * T[6 + e]));
  } else if (lane < 12) {
    const int d = lane - 9;
    const float c = d == 0 ? cx : (d == 1 ? cy : cz);
    v = fmaf(Ra[3 * d], T[9] - cx, fmaf(Ra[3 * d + 1], T[10] - cy, fmaf(Ra[3 * d + 2], T[11] - cz, c)));
  }
  if (lane < 12) A.item_orient[12 * (size_t)item + lane] = v;
  if (lane == 0) A.item_align[item] = (int16_t)a;
}

}  // namespace

hipError_t enqueue_align(const AlignArgs &A, int maxn, hipStream_t st) {
  const int64_t items = (int64_t)A.lig.n_ligands * A.n_orient;
  for (int64_t i0 = 0; i0 < items; i0 += kAlignChunk) {
    const int64_t m = items - i0 < kAlignChunk ? items - i0 : kAlignChunk;
    const dim3 grid((unsigned)((m + kAlignWaves - 1) / kAlignWaves)), block(kAlignWaves * kWave);
    if (maxn <= 64)
      hipLaunchKernelGGL(align_kernel<64>, grid, block, 0, st, A, i0, items);
    else if (maxn <= 128)
      hipLaunchKernelGGL(align_kernel<128>, grid, block, 0, st, A, i0, items);
    else
      hipLaunchKernelGGL(align_kernel<256>, grid, block, 0, st, A, i0, items);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace dock
