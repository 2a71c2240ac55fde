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
#include "rotamer_step.h"

namespace dock {

template <int WAVES, int TG>
__global__ void __launch_bounds__(WAVES *kWave)
    sweep_pruned_kernel(SweepArgs A, int nmax) {
  extern __shared__ float4 dyn_lds[];
  const int wv = threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  const WaveLds W((char *)dyn_lds + (size_t)wv * wave_lds_bytes(nmax), nmax);
  const GridView G = A.grid;
  const GridScaled GS = grid_scaled(G);
  const __amdgpu_buffer_rsrc_t grsrc = grid_rsrc(G);
  const int O = A.n_orient, S = A.S;
  const int T = (S + kWave - 1) / kWave;
  const float r2 = A.r2;
  const float thr = r2 + kPruneMargin;
  const bool emit = A.emit_x != nullptr;  // profile emission: S == 256, TG == 4
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
    stage_pose(W, G, A.lig.xyz + 3 * (size_t)a0, n, A.orient + 12 * o, lane);

    const size_t kbase = ((size_t)r0 * O + (size_t)o * R) * A.passes;
    int16_t *kout = A.kstar + kbase;
    int step = 0;
    int kreg = -1;  // lane s holds the choice of step s (mod 64) until written out
    for (int pass = 0; pass < A.passes; ++pass) {
      for (int r = 0; r < R; ++r, ++step) {
        const int ms = A.lig.move_offset[r0 + r];
        const RotState RS = rotamer_setup(W, n, A.lig.rot_axis[2 * (r0 + r)],
                                          A.lig.rot_axis[2 * (r0 + r) + 1],
                                          A.lig.move_atoms + ms,
                                          A.lig.move_offset[r0 + r + 1] - ms, lane);
        const float s0 = rotamer_s0(W, RS);
        if (emit) A.emit_x[(kbase + step) * 64 + lane] = f32_to_bf16(rotamer_feature(W, RS, G, lane));

        // invalid steps of the rotamer, for all S steps at once
        pair_tests += (uint64_t)rotamer_bump_mask(W, RS, r2, thr, S, lane);

        uint64_t best = 0ull;
        for (int t0 = 0; t0 < T; t0 += TG) {
          uint32_t bump = 0;
#pragma unroll
          for (int t = 0; t < TG; ++t) {
            const int k = (t0 + t) * kWave + lane;
            if (t0 + t >= T || k >= S || step_bumps(W, k)) bump |= 1u << t;
          }
          if (!emit) {
            const uint64_t key =
                best_valid_step<TG>(W, RS, G, GS, grsrc, A.cs, bump, t0, s0, lane);
            best = key > best ? key : best;
            continue;
          }
          // profile emission scores every step, valid or not
          float cc[TG], ss[TG], score[TG];
#pragma unroll
          for (int t = 0; t < TG; ++t) {
            const int k = (t0 + t) * kWave + lane;
            const float2 cs = A.cs[(t0 + t < T && k < S) ? k : 0];
            cc[t] = cs.x;
            ss[t] = cs.y;
          }
          rotamer_scores<TG>(W, RS, G, GS, grsrc, cc, ss, score, lane);
          if (t0 == 0 && lane == 0) score[0] = s0;
#pragma unroll
          for (int t = 0; t < TG; ++t) {
            const int k = (t0 + t) * kWave + lane;
            const uint64_t key = (bump >> t) & 1u ? 0ull : best_key(score[t], (uint32_t)k);
            best = key > best ? key : best;
          }
          float smax = score[0];
#pragma unroll
          for (int t = 1; t < TG; ++t) smax = fmaxf(smax, score[t]);
          smax = wave_max_f(smax);
          uint16_t *trow = A.emit_t + (kbase + step) * 256;
#pragma unroll
          for (int t = 0; t < TG; ++t) {
            trow[(t0 + t) * kWave + lane] = f32_to_bf16(fmaxf(score[t] - smax, -4.0f));
            const uint64_t vm = __ballot(!((bump >> t) & 1u));
            if (lane < 2)
              A.emit_mask[(kbase + step) * 8 + (t0 + t) * 2 + lane] = (uint32_t)(vm >> (32 * lane));
          }
        }
        best = wave_max_u64(best);
        const int kb = best ? (int)key_index(best) : -1;
        if (lane == (step & 63)) kreg = kb;
        if ((step & 63) == 63) kout[(step & ~63) + lane] = (int16_t)kreg;
        if (kb > 0) {
          const float2 cs = A.cs[kb];
          rotamer_apply(W, RS, G, cs.x, cs.y, lane);
        }
      }
    }
    if ((step & 63) != 0 && lane < (step & 63)) kout[(step & ~63) + lane] = (int16_t)kreg;
    float total = 0.0f;
    for (int i = lane; i < n; i += kWave) total += W.X[i].w;
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
  const size_t shmem = (size_t)WAVES * wave_lds_bytes(nmax);
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
