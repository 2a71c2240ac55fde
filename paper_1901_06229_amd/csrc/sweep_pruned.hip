// Greedy rotamer sweep with the bump test reduced to the pairs that can clash.
//
// Same mapping as the direct kernel (one 64-lane wave per (ligand,
// orientation) item, persistent grid, work stealing; lanes = angle steps),
// but the per-rotamer work is restructured around the rotation's geometry:
//
//   * Every atom is written once per rotamer in cylindrical form about the
//     bond axis (radial vector r, axial z).  A moving atom at angle theta is
//     a + z u + cos(theta) r + sin(theta) (u x r): 6 FMAs per angle.
//   * For a cross pair (i moving, j static) the squared distance at angle
//     theta is  d^2 = D' - 2 (cos(theta) A + sin(theta) B)  with
//     A = r_i.r_j, B = u.(r_i x r_j), D' = |r_i|^2 + |r_j|^2 + (z_i - z_j)^2,
//     and it never drops below (|r_i| - |r_j|)^2 + (z_i - z_j)^2.  Pairs whose
//     lower bound clears r_bump^2 (plus a margin far above FP32 rounding)
//     can never bump and are dropped; only the rest -- a few percent of
//     the cross pairs -- are tested, at 2 FMAs and a compare per angle.
//   * Survivors are compacted with ballots into an LDS list that every lane
//     (angle) walks; the scores are gathered per angle in atom order.
// The pair test is d^2 < r_bump^2 exactly as in the direct form; only the
// algebra that evaluates d^2 differs (FP32 rounding at the 1e-6 A level).
#include <hip/hip_runtime.h>

#include "dock_internal.h"
#include "sweep_common.h"

// Build-time choice of the scoring loop (same results either way):
//   DOCK_GATHER_ATOMS: moving atoms whose gathers are issued together (1, 2).
#ifndef DOCK_GATHER_ATOMS
#define DOCK_GATHER_ATOMS 1
#endif

namespace dock {

constexpr int kPairCap = 128;  // LDS pair-list entries per wave

__host__ __device__ inline int pruned_head_bytes(int nmax) {
  // X, C (float4), rho (float), Q, M (int16), mov (uint8)
  const int b = nmax * 16 * 2 + nmax * 4 + nmax * 2 * 2 + nmax;
  return (b + 15) / 16 * 16;
}

__host__ __device__ inline int pruned_wave_bytes(int nmax) {
  // then the pair list: coefficients (float4) and packed atom pairs (int32)
  return pruned_head_bytes(nmax) + kPairCap * (16 + 4);
}

template <int WAVES, int TG>
__global__ void __launch_bounds__(WAVES *kWave)
    sweep_pruned_kernel(SweepArgs A, int nmax) {
  extern __shared__ float4 dyn_lds[];
  const int wv = threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  char *wbase = (char *)dyn_lds + (size_t)wv * pruned_wave_bytes(nmax);
  float4 *X = (float4 *)wbase;                 // pose: x, y, z, voxel value
  float4 *C = X + nmax;                        // cylinder coords about the axis
  float *rho = (float *)(C + nmax);            // |r|
  int16_t *Q = (int16_t *)(rho + nmax);        // static cross set
  int16_t *M = Q + nmax;                       // moving set of the rotamer
  uint8_t *mov = (uint8_t *)(M + nmax);
  float4 *P = (float4 *)(wbase + pruned_head_bytes(nmax));  // kept pairs: 2A, 2B, D
  int *PI = (int *)(P + kPairCap);                           // kept pairs: i << 16 | j

  const GridView G = A.grid;
  const GridScaled GS = grid_scaled(G);
  const __amdgpu_buffer_rsrc_t grsrc = grid_rsrc(G);
  const int O = A.n_orient, S = A.S;
  const int T = (S + kWave - 1) / kWave;
  const float r2 = A.r2;
  const float thr = r2 + kPruneMargin;
  const uint64_t lanes_below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint64_t pair_tests = 0;  // executed (pair, angle) tests of this wave

  int cur = 0, end = 0;  // items claimed by this wave, [cur, end)
  for (;;) {
    if (cur >= end) {
      int base = 0;
      if (lane == 0) base = atomicAdd(A.queue, A.claim);
      base = __shfl(base, 0, kWave);
      base = __builtin_amdgcn_readfirstlane(base);
      if (base >= A.n_items) break;
      cur = base;
      end = min(base + A.claim, A.n_items);
    }
    const int item = cur++;
    const int slot = item / O;
    const int o = item - slot * O;
    const int l = A.order[slot];
    if (A.status[l] != 0) continue;
    const int a0 = A.lig.atom_offset[l];
    const int n = A.lig.atom_offset[l + 1] - a0;
    const int r0 = A.lig.rot_offset[l];
    const int R = A.lig.rot_offset[l + 1] - r0;
    const float *Tr = A.orient + 12 * o;

    for (int i = lane; i < n; i += kWave) {
      const float *p = A.lig.xyz + 3 * (size_t)(a0 + i);
      float3 x = orient_point(Tr, p[0], p[1], p[2]);
      X[i] = make_float4(x.x, x.y, x.z, voxel_value(G, x.x, x.y, x.z));
    }
    wave_lds_sync();

    int16_t *kout = A.kstar + ((size_t)r0 * O + (size_t)o * R) * A.passes;
    int step = 0;
    int kreg = -1;  // lane s holds the choice of step s (mod 64) until written out
    for (int pass = 0; pass < A.passes; ++pass) {
      for (int r = 0; r < R; ++r, ++step) {
        const int ra = A.lig.rot_axis[2 * (r0 + r)];
        const int rb = A.lig.rot_axis[2 * (r0 + r) + 1];
        const int ms = A.lig.move_offset[r0 + r];
        const int m = A.lig.move_offset[r0 + r + 1] - ms;
        const int16_t *mlist = A.lig.move_atoms + ms;
        for (int i = lane; i < n; i += kWave) mov[i] = 0;
        wave_lds_sync();
        for (int t = lane; t < m; t += kWave) {
          const int i = mlist[t];
          mov[i] = 1;
          M[t] = (int16_t)i;
        }
        wave_lds_sync();
        int q = 0;
        for (int base = 0; base < n; base += kWave) {
          const int i = base + lane;
          const bool st = i < n && !mov[i] && i != ra && i != rb;
          const uint64_t mask = __ballot(st);
          if (st) Q[q + __popcll(mask & lanes_below)] = (int16_t)i;
          q += __popcll(mask);
        }
        // score of everything that does not move: per-lane partial sums in
        // atom order, then a fixed butterfly over the wave
        float cst = 0.0f;
        for (int i = lane; i < n; i += kWave)
          if (!mov[i]) cst += X[i].w;
        cst = wave_sum(cst);
        const float4 xa = X[ra];
        const float3 u = bond_axis(xa, X[rb]);
        for (int i = lane; i < n; i += kWave) {
          Cyl c = cyl_of(X[i], xa, u);
          C[i] = make_float4(c.rx, c.ry, c.rz, c.z);
          rho[i] = sqrtf(fmaf(c.rx, c.rx, fmaf(c.ry, c.ry, c.rz * c.rz)));
        }
        wave_lds_sync();

        // exact score of the current pose (angle step 0), in atom order
        float s0 = cst;
        for (int tm = 0; tm < m; ++tm) s0 += X[M[tm]].w;

        uint64_t best = 0ull;
        for (int t0 = 0; t0 < T; t0 += TG) {
          float cc[TG], ss[TG], score[TG];
          uint32_t bump = 0;
#pragma unroll
          for (int t = 0; t < TG; ++t) {
            const int k = (t0 + t) * kWave + lane;
            const bool act = (t0 + t < T) && k < S;
            const float2 cs = A.cs[act ? k : 0];
            cc[t] = cs.x;
            ss[t] = cs.y;
            score[t] = cst;
            if (!act) bump |= 1u << t;
          }
          const int S_grp = min(S, (t0 + TG) * kWave) - t0 * kWave;
          // -- bump test.  Lanes sweep the flattened cross pairs (i in M, j in
          // Q) and keep those whose lower bound does not clear r_bump; the
          // kept pairs get their harmonic coefficients, and every lane
          // (angle) then tests them.
          auto test_pairs = [&](int cnt) {
            pair_tests += (uint64_t)cnt * (uint64_t)S_grp;
            for (int e = lane; e < cnt; e += kWave) {
              const int ij = PI[e];
              const float4 ci = C[ij >> 16], cj = C[ij & 0xFFFF];
              const float dz = ci.w - cj.w;
              const float a_ = fmaf(ci.x, cj.x, fmaf(ci.y, cj.y, ci.z * cj.z));
              const float cx = ci.y * cj.z - ci.z * cj.y;
              const float cy = ci.z * cj.x - ci.x * cj.z;
              const float cz = ci.x * cj.y - ci.y * cj.x;
              const float b_ = fmaf(u.x, cx, fmaf(u.y, cy, u.z * cz));
              const float rho2i = fmaf(ci.x, ci.x, fmaf(ci.y, ci.y, ci.z * ci.z));
              const float rho2j = fmaf(cj.x, cj.x, fmaf(cj.y, cj.y, cj.z * cj.z));
              P[e] = make_float4(2.0f * a_, 2.0f * b_, fmaf(dz, dz, rho2i + rho2j) - r2, 0.0f);
            }
            wave_lds_sync();
            for (int e = 0; e < cnt; ++e) {
              const float4 pr = P[e];
#pragma unroll
              for (int t = 0; t < TG; ++t)
                if (fmaf(cc[t], pr.x, ss[t] * pr.y) > pr.z) bump |= 1u << t;
            }
            wave_lds_sync();
          };
          {
            const int total = m * q;
            const float inv_q = q > 0 ? 1.0f / (float)q : 0.0f;
            int np = 0;
            for (int base = 0; base < total; base += kWave) {
              const int pidx = base + lane;
              bool act = false;
              int packed = 0;
              if (pidx < total) {
                int ii = (int)(((float)pidx + 0.5f) * inv_q);
                int jj = pidx - ii * q;
                if (jj < 0) { --ii; jj += q; }
                if (jj >= q) { ++ii; jj -= q; }
                const int i = M[ii], j = Q[jj];
                const float dz = C[i].w - C[j].w;
                const float dr = rho[i] - rho[j];
                act = fmaf(dr, dr, dz * dz) < thr;
                packed = (i << 16) | j;
              }
              const uint64_t mask = __ballot(act);
              if (act) PI[np + __popcll(mask & lanes_below)] = packed;
              np += __popcll(mask);
              if (np > kPairCap - kWave) {
                wave_lds_sync();
                test_pairs(np);
                np = 0;
              }
            }
            wave_lds_sync();
            test_pairs(np);
          }
          // -- scores of the angles that survived, gathered in atom order.
          // Lanes hold the voxel-space rotation basis of up to 64 moving atoms
          // ((p - o)/h, e/h, f/h); every lane reads one atom's basis at a time
          // and issues the gathers of all its angle tiles before using any.
          const uint32_t full = (TG >= 32) ? 0xFFFFFFFFu : ((1u << TG) - 1u);
          if (__ballot(bump != full) != 0ull) {
            for (int c0 = 0; c0 < m; c0 += kWave) {
              float b0 = 0.f, b1 = 0.f, b2 = 0.f, b3 = 0.f, b4 = 0.f, b5 = 0.f, b6 = 0.f,
                    b7 = 0.f, b8 = 0.f;
              if (c0 + lane < m) {
                const float4 ci = C[M[c0 + lane]];
                const RotBasis bs = rot_basis(Cyl{ci.x, ci.y, ci.z, ci.w}, xa, u);
                b0 = (bs.px - G.ox) * G.inv_h;
                b1 = (bs.py - G.oy) * G.inv_h;
                b2 = (bs.pz - G.oz) * G.inv_h;
                b3 = bs.ex * G.inv_h;
                b4 = bs.ey * G.inv_h;
                b5 = bs.ez * G.inv_h;
                b6 = bs.fx * G.inv_h;
                b7 = bs.fy * G.inv_h;
                b8 = bs.fz * G.inv_h;
              }
              const int cnt = min(kWave, m - c0);
              // two atoms per iteration: all 2 TG gathers are in flight before
              // the first is used; sums stay in atom order
              int tt = 0;
              for (; DOCK_GATHER_ATOMS == 2 && tt + 1 < cnt; tt += 2) {
                uint32_t off[2][TG];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                  const float px = lane_bcast(b0, tt + h), py = lane_bcast(b1, tt + h),
                              pz = lane_bcast(b2, tt + h), ex = lane_bcast(b3, tt + h),
                              ey = lane_bcast(b4, tt + h), ez = lane_bcast(b5, tt + h),
                              fx = lane_bcast(b6, tt + h), fy = lane_bcast(b7, tt + h),
                              fz = lane_bcast(b8, tt + h);
#pragma unroll
                  for (int t = 0; t < TG; ++t)
                    off[h][t] = voxel_byte_offset(GS, fmaf(ss[t], fx, fmaf(cc[t], ex, px)),
                                                  fmaf(ss[t], fy, fmaf(cc[t], ey, py)),
                                                  fmaf(ss[t], fz, fmaf(cc[t], ez, pz)));
                }
                float val[2][TG];
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                  for (int t = 0; t < TG; ++t) val[h][t] = grid_load(grsrc, off[h][t]);
#pragma unroll
                for (int t = 0; t < TG; ++t) score[t] = (score[t] + val[0][t]) + val[1][t];
              }
              for (; tt < cnt; ++tt) {
                const float px = lane_bcast(b0, tt), py = lane_bcast(b1, tt), pz = lane_bcast(b2, tt);
                const float ex = lane_bcast(b3, tt), ey = lane_bcast(b4, tt), ez = lane_bcast(b5, tt);
                const float fx = lane_bcast(b6, tt), fy = lane_bcast(b7, tt), fz = lane_bcast(b8, tt);
                uint32_t off[TG];
#pragma unroll
                for (int t = 0; t < TG; ++t)
                  off[t] = voxel_byte_offset(GS, fmaf(ss[t], fx, fmaf(cc[t], ex, px)),
                                             fmaf(ss[t], fy, fmaf(cc[t], ey, py)),
                                             fmaf(ss[t], fz, fmaf(cc[t], ez, pz)));
                float val[TG];
#pragma unroll
                for (int t = 0; t < TG; ++t) val[t] = grid_load(grsrc, off[t]);
#pragma unroll
                for (int t = 0; t < TG; ++t) score[t] += val[t];
              }
            }
          }
          if (t0 == 0 && lane == 0) score[0] = s0;
#pragma unroll
          for (int t = 0; t < TG; ++t) {
            const int k = (t0 + t) * kWave + lane;
            const uint64_t key = (bump >> t) & 1u ? 0ull : best_key(score[t], (uint32_t)k);
            best = key > best ? key : best;
          }
        }
        best = wave_max_u64(best);
        const int kb = best ? (int)key_index(best) : -1;
        if (lane == (step & 63)) kreg = kb;
        if ((step & 63) == 63) kout[(step & ~63) + lane] = (int16_t)kreg;
        if (kb > 0) {
          const float2 cs = A.cs[kb];
          for (int t = lane; t < m; t += kWave) {
            const int i = mlist[t];
            const float4 ci = C[i];
            const RotBasis bs = rot_basis(Cyl{ci.x, ci.y, ci.z, ci.w}, xa, u);
            const float3 y = rot_apply(bs, cs.x, cs.y);
            X[i] = make_float4(y.x, y.y, y.z, voxel_value(G, y.x, y.y, y.z));
          }
        }
        wave_lds_sync();
      }
    }
    if ((step & 63) != 0 && lane < (step & 63)) kout[(step & ~63) + lane] = (int16_t)kreg;
    float total = 0.0f;
    for (int i = lane; i < n; i += kWave) total += X[i].w;
    total = wave_sum(total);
    if (lane == 0) {
      if (A.all_scores) A.all_scores[(size_t)l * O + o] = total;
      atomicMax(A.keys + l, (unsigned long long)best_key(total, (uint32_t)o));
    }
    wave_lds_sync();
  }
  if (lane == 0 && A.pair_tests) atomicAdd(A.pair_tests, (unsigned long long)pair_tests);
}

template <int WAVES, int TG>
static hipError_t launch_pruned_t(const SweepArgs &A, int nmax, int blocks_per_cu, int n_cu,
                                  hipStream_t st) {
  const size_t shmem = (size_t)WAVES * pruned_wave_bytes(nmax);
  if (shmem > 65536) return hipErrorInvalidValue;
  int occ = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &occ, sweep_pruned_kernel<WAVES, TG>, WAVES * kWave, shmem);
  if (e != hipSuccess) return e;
  if (occ < 1) occ = 1;
  const int bpc = blocks_per_cu > 0 && blocks_per_cu < occ ? blocks_per_cu : occ;
  const int64_t need = (A.n_items + WAVES - 1) / WAVES;
  int64_t grid = (int64_t)bpc * n_cu;
  if (grid > need) grid = need;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL((sweep_pruned_kernel<WAVES, TG>), dim3((unsigned)grid),
                     dim3(WAVES * kWave), shmem, st, A, nmax);
  return hipGetLastError();
}

template <int WAVES>
static hipError_t launch_pruned_w(const SweepArgs &A, int nmax, int blocks_per_cu, int n_cu,
                                  hipStream_t st) {
  const int T = (A.S + kWave - 1) / kWave;
  if (T <= 1) return launch_pruned_t<WAVES, 1>(A, nmax, blocks_per_cu, n_cu, st);
  if (T <= 2) return launch_pruned_t<WAVES, 2>(A, nmax, blocks_per_cu, n_cu, st);
  if (T <= 4) return launch_pruned_t<WAVES, 4>(A, nmax, blocks_per_cu, n_cu, st);
  if (T <= 6) return launch_pruned_t<WAVES, 6>(A, nmax, blocks_per_cu, n_cu, st);
  return launch_pruned_t<WAVES, 8>(A, nmax, blocks_per_cu, n_cu, st);
}

hipError_t enqueue_sweep_pruned(const SweepArgs &A, int max_atoms, const LaunchPlan &plan,
                                int n_cu, hipStream_t st) {
  if (A.n_items <= 0) return hipSuccess;
  const int nmax = (max_atoms + 15) / 16 * 16;
  switch (plan.waves_per_block) {
    case 1: return launch_pruned_w<1>(A, nmax, plan.blocks_per_cu, n_cu, st);
    case 2: return launch_pruned_w<2>(A, nmax, plan.blocks_per_cu, n_cu, st);
    case 4: return launch_pruned_w<4>(A, nmax, plan.blocks_per_cu, n_cu, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dock
