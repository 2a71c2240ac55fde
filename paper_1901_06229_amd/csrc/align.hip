// Rigid alignment search before the rotamer sweep (paper §3.1: the first
// phase treats the ligand as a rigid body and looks for the orientation that
// fits the pocket best, scoring every rotation; §4.1: rotation and scoring are
// fused so that no rotated pose is stored, a reduction picks the best
// orientation, and the ligand is rotated once).
//
// One block per ligand, one wave per (ligand, orientation) restart at a time,
// one lane per candidate rotation.  A restart's starting pose is staged in LDS
// as coordinates relative to its centroid, in voxel units; every lane reads
// the same atom at a time (an LDS broadcast), rotates it with its own matrix
// and accumulates voxel values.  A wave reduction over (score, index) keys
// selects the best rotation, lowest index on ties.  The winner is not applied
// to a pose: it is folded into the restart's rigid transform
//     X = R_a (R_o x + t_o - c) + c = (R_a R_o) x + (R_a (t_o - c) + c),
// which the sweep stages like any orientation.
//
// Voxel values: the 64 lanes send one atom to 64 scattered points on a sphere
// about the centroid, so a gather from the grid in global memory costs about
// one L2 cache line per lane.  The block therefore first copies a cube of
// grid values around the ligand's first restart into LDS (the voxels of
// indices lo .. lo + side - 1 per axis, clamped to the box as the score
// requires; the corner lo is kept at or above 0).  The image t of an atom, in
// voxel units, is computed the same way on either route; for t >= lo >= 0,
// t - lo is exact in FP32 (a non-negative integer no larger than t subtracted
// from t below 2^24), so a lane inside the cube reads exactly the voxel the
// global lookup would.  Atoms whose images
// provably stay inside the cube for every rotation (distance from the
// centroid times the largest row norm of the set, plus the centroid's offset
// from the cube centre, below half the side) take the LDS route without a
// test; for the others each lane tests its image and reads the cube or
// global memory.  Inner atoms are summed first, then outer atoms, each in
// atom order.
#include "dock_internal.h"

namespace dock {
namespace {

constexpr int kCubeHalf = 15;                   // cube of kCubeSide^3 voxels in LDS
constexpr int kCubeSide = 2 * kCubeHalf + 1;    // 31: 119,164 bytes
constexpr int kCubeVox = kCubeSide * kCubeSide * kCubeSide;
// margin (voxels) for FP32 rounding of the image coordinates
constexpr float kCubeMargin = 0.05f;
// ligands per launch: keeps the grid below 2^32 work-items per dimension
constexpr int kAlignLigChunk = 1 << 22;

// waves per block: as many as fit beside the cube (160 KB of LDS per CU)
template <int MAXN>
constexpr int align_waves() { return MAXN <= 128 ? 16 : 8; }

// Starting pose of restart o written to Z as centroid-relative coordinates in
// voxel units, inner atoms first (order kept within each class; w = 1 marks
// an inner atom).  Returns the number of inner atoms, the centroid c and the
// centroid in voxel units relative to the grid origin, q.
template <int MAXN>
__device__ __forceinline__ int stage_restart(const AlignArgs &A, float4 *Z, int a0, int n, int o,
                                             float rho, const float C[3], int lane, float3 &c,
                                             float &qx, float &qy, float &qz) {
  constexpr int kChunks = MAXN / kWave;
  const float *T = A.orient + 12 * (size_t)o;
  float3 x[kChunks];
  float sx = 0.0f, sy = 0.0f, sz = 0.0f;
#pragma unroll
  for (int k = 0; k < kChunks; ++k) {
    const int i = lane + k * kWave;
    x[k] = make_float3(0.0f, 0.0f, 0.0f);
    if (i < n) {
      const float *p = A.lig.xyz + 3 * (size_t)(a0 + i);
      x[k] = orient_point(T, p[0], p[1], p[2]);
      sx += x[k].x;
      sy += x[k].y;
      sz += x[k].z;
    }
  }
  // hardware reciprocal (about 1 ulp): the centroid is this kernel's own and
  // is folded into the composed transform it writes
  const float inv_n = __builtin_amdgcn_rcpf((float)n);
  const float cx = wave_sum(sx) * inv_n, cy = wave_sum(sy) * inv_n, cz = wave_sum(sz) * inv_n;
  c = make_float3(cx, cy, cz);
  const GridView &G = A.grid;
  const float ih = G.inv_h;
  qx = (cx - G.ox) * ih;
  qy = (cy - G.oy) * ih;
  qz = (cz - G.oz) * ih;
  const float off = fmaxf(fabsf(qx - C[0]), fmaxf(fabsf(qy - C[1]), fabsf(qz - C[2])));
  const float reach = (float)kCubeHalf + 0.5f - kCubeMargin - off;
  // inner / outer classification and a stable partition
  bool inner[kChunks];
  int n_inner = 0;
#pragma unroll
  for (int k = 0; k < kChunks; ++k) {
    const int i = lane + k * kWave;
    x[k] = make_float3((x[k].x - cx) * ih, (x[k].y - cy) * ih, (x[k].z - cz) * ih);
    // hardware square root: its ~1 ulp is far inside kCubeMargin
    const float r = __builtin_amdgcn_sqrtf(fmaf(x[k].x, x[k].x, fmaf(x[k].y, x[k].y, x[k].z * x[k].z)));
    inner[k] = i < n && rho * r <= reach;
    n_inner += __popcll(__ballot(inner[k]));
  }
  int seen_in = 0, seen_out = 0;
#pragma unroll
  for (int k = 0; k < kChunks; ++k) {
    const int i = lane + k * kWave;
    const uint64_t m_in = __ballot(inner[k]);
    const uint64_t m_out = __ballot(i < n && !inner[k]);
    if (i < n) {
      const int slot = inner[k] ? lanes_before(m_in, seen_in) : lanes_before(m_out, n_inner + seen_out);
      Z[slot] = make_float4(x[k].x, x[k].y, x[k].z, inner[k] ? 1.0f : 0.0f);
    }
    seen_in += __popcll(m_in);
    seen_out += __popcll(m_out);
  }
  wave_lds_sync();
  return n_inner;
}

template <int MAXN>
__global__ void __launch_bounds__(align_waves<MAXN>() * kWave)
    align_kernel(AlignArgs A, int l0) {
  constexpr int WAVES = align_waves<MAXN>();
  __shared__ float sCube[kCubeVox];
  __shared__ float4 sZ[WAVES][MAXN];
  const int l = l0 + (int)blockIdx.x;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  const int lane = threadIdx.x % kWave;
  const int O = A.n_orient;
  if (A.status[l] != 0) {  // uniform over the block
    for (int o = threadIdx.x; o < O; o += WAVES * kWave) A.item_align[(size_t)l * O + o] = -1;
    return;
  }
  const int a0 = A.lig.atom_offset[l];
  const int n = A.lig.atom_offset[l + 1] - a0;  // 1 .. MAXN once validated
  const GridView G = A.grid;
  float4 *Z = sZ[wv];

  // largest row norm over the rotation set (1 for rotations): bounds |R z| by rho |z|
  float rho_l = 0.0f;
  for (int a = lane; a < A.n_align; a += kWave) {
    const float *Rm = A.rot + 9 * (size_t)a;
#pragma unroll
    for (int d = 0; d < 3; ++d)
      rho_l = fmaxf(rho_l, sqrtf(fmaf(Rm[3 * d], Rm[3 * d], fmaf(Rm[3 * d + 1], Rm[3 * d + 1],
                                                                 Rm[3 * d + 2] * Rm[3 * d + 2]))));
  }
  const float rho = wave_max_f(rho_l) * (1.0f + 1e-6f);

  // cube around the first restart's centroid (every wave derives the same corner)
  float q0x, q0y, q0z;
  {
    const float far[3] = {3.0e38f, 3.0e38f, 3.0e38f};  // classifies every atom as outer
    float3 c0;
    stage_restart<MAXN>(A, Z, a0, n, 0, rho, far, lane, c0, q0x, q0y, q0z);
  }
  // a corner below 0 would make t - lo an addition, which can round up
  // across a face; clamped cells past the far border are read as stored
  const int lox = max((int)floorf(q0x) - kCubeHalf, 0), loy = max((int)floorf(q0y) - kCubeHalf, 0),
            loz = max((int)floorf(q0z) - kCubeHalf, 0);
  const float C[3] = {(float)lox + 0.5f * kCubeSide, (float)loy + 0.5f * kCubeSide,
                      (float)loz + 0.5f * kCubeSide};
  for (int v = threadIdx.x; v < kCubeVox; v += WAVES * kWave) {
    const int lx = v % kCubeSide, ly = (v / kCubeSide) % kCubeSide, lz = v / (kCubeSide * kCubeSide);
    const int gx = min(max(lox + lx, 0), G.nx - 1), gy = min(max(loy + ly, 0), G.ny - 1),
              gz = min(max(loz + lz, 0), G.nz - 1);
    sCube[v] = G.grid[((size_t)gz * G.ny + gy) * G.nx + gx];
  }
  __syncthreads();

  const GridScaled GS = grid_scaled(G);
  const __amdgpu_buffer_rsrc_t grsrc = grid_rsrc(G);
  for (int o = wv; o < O; o += WAVES) {
    float qx, qy, qz;
    float3 c;
    const int ni = stage_restart<MAXN>(A, Z, a0, n, o, rho, C, lane, c, qx, qy, qz);
    const float flx = (float)lox, fly = (float)loy, flz = (float)loz, fside = (float)kCubeSide;
    uint64_t best = 0;
    for (int c0 = 0; c0 < A.n_align; c0 += kWave) {
      const int a = c0 + lane;
      const float *Rm = A.rot + 9 * (size_t)min(a, A.n_align - 1);
      const float m0 = Rm[0], m1 = Rm[1], m2 = Rm[2], m3 = Rm[3], m4 = Rm[4], m5 = Rm[5],
                  m6 = Rm[6], m7 = Rm[7], m8 = Rm[8];
      float s = 0.0f;
#pragma unroll 4
      for (int i = 0; i < ni; ++i) {  // images inside the cube for every rotation
        const float4 z = Z[i];
        const float tx = fmaf(m0, z.x, fmaf(m1, z.y, fmaf(m2, z.z, qx)));
        const float ty = fmaf(m3, z.x, fmaf(m4, z.y, fmaf(m5, z.z, qy)));
        const float tz = fmaf(m6, z.x, fmaf(m7, z.y, fmaf(m8, z.z, qz)));
        const uint32_t lx = (uint32_t)(tx - flx), ly = (uint32_t)(ty - fly), lz = (uint32_t)(tz - flz);
        s += sCube[__umul24(__umul24(lz, kCubeSide) + ly, kCubeSide) + lx];
      }
#pragma unroll 2
      for (int i = ni; i < n; ++i) {  // each lane tests its own image
        const float4 z = Z[i];
        const float tx = fmaf(m0, z.x, fmaf(m1, z.y, fmaf(m2, z.z, qx)));
        const float ty = fmaf(m3, z.x, fmaf(m4, z.y, fmaf(m5, z.z, qy)));
        const float tz = fmaf(m6, z.x, fmaf(m7, z.y, fmaf(m8, z.z, qz)));
        const float ex = tx - flx, ey = ty - fly, ez = tz - flz;
        float v;
        if (ex >= 0.0f && ex < fside && ey >= 0.0f && ey < fside && ez >= 0.0f && ez < fside)
          v = sCube[__umul24(__umul24((uint32_t)ez, kCubeSide) + (uint32_t)ey, kCubeSide) + (uint32_t)ex];
        else
          v = grid_load(grsrc, voxel_byte_offset(GS, tx, ty, tz));
        s += v;
      }
      if (a < A.n_align) {
        const uint64_t k = best_key(s, (uint32_t)a);
        best = k > best ? k : best;
      }
    }
    best = wave_max_u64(best);
    const int a = (int)key_index(best);

    // fold the winner into the restart's transform: lanes 0-8 the matrix
    // entries, lanes 9-11 the translation
    const float *T = A.orient + 12 * (size_t)o;
    const float cx = c.x, cy = c.y, cz = c.z;
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
    const size_t item = (size_t)l * O + o;
    if (lane < 12) A.item_orient[12 * item + lane] = v;
    if (lane == 0) A.item_align[item] = (int16_t)a;
    wave_lds_sync();  // Z is restaged for the next restart
  }
}

}  // namespace

hipError_t enqueue_align(const AlignArgs &A, int maxn, hipStream_t st) {
  const int L = A.lig.n_ligands;
  for (int l0 = 0; l0 < L; l0 += kAlignLigChunk) {
    const dim3 grid((unsigned)min(kAlignLigChunk, L - l0));
    if (maxn <= 64)
      hipLaunchKernelGGL(align_kernel<64>, grid, dim3(align_waves<64>() * kWave), 0, st, A, l0);
    else if (maxn <= 128)
      hipLaunchKernelGGL(align_kernel<128>, grid, dim3(align_waves<128>() * kWave), 0, st, A, l0);
    else
      hipLaunchKernelGGL(align_kernel<256>, grid, dim3(align_waves<256>() * kWave), 0, st, A, l0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace dock
