// Greedy rotamer sweep with the bump test reduced to the pairs that can clash.
//
// One 64-lane wave per (ligand, orientation) item, persistent grid, items
// taken from a cost-sorted queue by guided claims.  Per rotamer step the wave
// handles all S angle steps at once, restructured around the rotation's
// geometry:
//
//   * Every atom is written once per step in cylindrical form about the bond
//     axis (radial vector r, axial z).  A moving atom at angle theta is
//     a + z u + cos(theta) r + sin(theta) (u x r): 6 FMAs per angle.
//   * A cross pair (i moving, j static) has squared distance
//     d^2 = D' - 2 (cos(theta) A + sin(theta) B) with A = r_i.r_j,
//     B = u.(r_i x r_j), D' = |r_i|^2 + |r_j|^2 + (z_i - z_j)^2, never below
//     (|r_i| - |r_j|)^2 + (z_i - z_j)^2.  Pairs whose bound clears r_bump^2
//     (plus a margin far above FP32 rounding) can never bump and are dropped.
//   * Each kept pair bumps on one open arc of angles, found in closed form
//     and marked into a bitmask of all S steps; only the non-bumping steps
//     are then scored, compacted into full 64-lane tiles, with the gathers
//     added in atom order.
// The pair test is d^2 < r_bump^2 as in the direct form; only the algebra
// that decides it differs (FP32 rounding at the 1e-6 A level).
#include <hip/hip_runtime.h>

#include "dock_internal.h"
#include "sweep_common.h"
#include "rotamer_step.h"

namespace dock {

// LB: the moving atoms' rotation bases are staged in LDS for the scoring
// loop (chosen at launch when the extra LDS costs no occupancy).  EMIT: the
// profile-emission form (every angle scored, features and landscapes
// written), a separate instantiation so the plain sweep does not carry its
// registers.
template <int WAVES, int TG, bool LB, bool EMIT>
__global__ void __launch_bounds__(WAVES *kWave)
    sweep_pruned_kernel(SweepArgs args, int nmax) {
  // Fields are read from the kernel-argument segment (constant memory, the
  // struct at offset 0) at their uses: the compiler reloads such invariant
  // scalars instead of spilling them to vector-register lanes (about a
  // hundred fewer spill moves in the code, 0.8 % fewer VALU instructions
  // executed per rotamer step).
  (void)args;
  const SweepArgs &A = *(const SweepArgs *)__builtin_amdgcn_kernarg_segment_ptr();
  extern __shared__ float4 dyn_lds[];
  const int wv = threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  const WaveLds W((char *)dyn_lds + (size_t)wv * wave_lds_bytes(nmax, LB, TG, A.S), nmax, LB, TG);
  const GridView G = A.grid;
  const GridScaled GS = grid_scaled(G);
  const __amdgpu_buffer_rsrc_t grsrc = grid_rsrc(G);
  const int O = A.n_orient, S = A.S;
  const int T = (S + kWave - 1) / kWave;
  const float r2 = A.r2;
  const int thr_q = zr_threshold(r2 + kPruneMargin);
  constexpr bool emit = EMIT;  // profile emission: S == 256, TG == 4
  uint64_t kept_pairs = 0, evals = 0;  // work counters of this wave

  // the last size class: slots [cb, ce) of the cost order (all of them when
  // no grouped class is in use)
  const int cb = A.small[kClassBegin + kClasses - 1], ce = A.small[kClassEnd + kClasses - 1];
  WorkQueue queue(A.queue, (ce - cb) * O, A.claim, (int)gridDim.x * WAVES);
  for (int item; queue.next(lane, item);) {
    const int slot = cb + item / O;
    const int o = item - (slot - cb) * O;
    const int l = A.order[slot];
    if (A.status[l] != 0) continue;
    const int a0 = A.lig.atom_offset[l];
    const int n = A.lig.atom_offset[l + 1] - a0;
    const int r0 = A.lig.rot_offset[l];
    const int R = A.lig.rot_offset[l + 1] - r0;
    stage_pose(W, G, A.lig.xyz + 3 * (size_t)a0, n, A.orient + 12 * ((size_t)l * A.orient_stride + o), lane);

    const size_t kbase = ((size_t)r0 * O + (size_t)o * R) * A.passes;
    int16_t *kout = A.kstar + kbase;
    const int steps = R * A.passes;
    int step = 0;
    int kreg = -1;  // lane s holds the choice of step s (mod 64) until written out
    // topology of the current step; the next step's is fetched during it
    RotTopo topo{};
    if (steps > 0) topo = topo_finish(A.lig, topo_words_load(A.lig, r0, lane), lane);
    for (int pass = 0; pass < A.passes; ++pass) {
      for (int r = 0; r < R; ++r, ++step) {
        const bool more = step + 1 < steps;
        const int words_next = more ? topo_words_load(A.lig, r0 + (r + 1 == R ? 0 : r + 1), lane) : 0;
        const RotState RS = rotamer_setup(W, n, topo, A.lig.move_atoms, lane);
        const float s0 = rotamer_s0(W, RS, lane);
        if constexpr (emit)
          A.emit_x[(kbase + step) * 64 + lane] = f32_to_bf16(rotamer_feature(W, RS, G, lane));

        // invalid steps of the rotamer, for all S steps at once
        kept_pairs += (uint64_t)rotamer_bump_mask(W, RS, r2, thr_q, S, lane);
        const RotTopo topo_next = more ? topo_finish(A.lig, words_next, lane) : topo;

        uint64_t best = 0ull;
        for (int t0 = 0; t0 < T; t0 += TG) {
          uint64_t vm[TG];  // wave-uniform valid masks of the group's tiles
#pragma unroll
          for (int t = 0; t < TG; ++t) vm[t] = tile_valid_mask(W, t0 + t, S);
          if constexpr (!emit) {
            int nvalid;
            const uint64_t key =
                best_valid_step<TG, LB>(W, RS, G, GS, grsrc, A.cs, vm, t0, s0, lane, nvalid);
            best = key > best ? key : best;
            evals += (uint64_t)RS.m * (uint64_t)nvalid;
          } else {
            // profile emission scores every step, valid or not
            evals += (uint64_t)RS.m * (uint64_t)(TG * kWave);
            float cc[TG], ss[TG], score[TG];
#pragma unroll
            for (int t = 0; t < TG; ++t) {
              const int k = (t0 + t) * kWave + lane;
              const float2 cs = A.cs[(t0 + t < T && k < S) ? k : 0];
              cc[t] = cs.x;
              ss[t] = cs.y;
            }
            rotamer_scores<TG, LB>(W, RS, G, GS, grsrc, cc, ss, score, lane);
            if (t0 == 0 && lane == 0) score[0] = s0;
#pragma unroll
            for (int t = 0; t < TG; ++t) {
              const int k = (t0 + t) * kWave + lane;
              const uint64_t key = (vm[t] >> lane) & 1ull ? best_key(score[t], (uint32_t)k) : 0ull;
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
              if (lane < 2)
                A.emit_mask[(kbase + step) * 8 + (t0 + t) * 2 + lane] =
                    (uint32_t)(vm[t] >> (32 * lane));
            }
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
        topo = topo_next;
      }
    }
    if ((step & 63) != 0 && lane < (step & 63)) kout[(step & ~63) + lane] = (int16_t)kreg;
    const float total = pose_total(W, n, lane);
    if (lane == 0) {
      if (A.all_scores) A.all_scores[(size_t)l * O + o] = total;
      atomicMax(A.keys + l, (unsigned long long)best_key(total, (uint32_t)o));
    }
    wave_lds_sync();
  }
  if (lane == 0 && A.work) {
    atomicAdd(A.work, (unsigned long long)kept_pairs);
    atomicAdd(A.work + 1, (unsigned long long)evals);
  }
}

// Resident blocks per CU of one instantiation (0: its LDS exceeds a block's).
template <int WAVES, int TG, bool LB, bool EMIT = false>
static hipError_t pruned_occupancy(int nmax, int S, int blocks_per_cu, int *bpc) {
  *bpc = 0;
  const size_t shmem = (size_t)WAVES * wave_lds_bytes(nmax, LB, TG, S);
  if (shmem > 65536) return hipSuccess;
  int occ = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &occ, sweep_pruned_kernel<WAVES, TG, LB, EMIT>, WAVES * kWave, shmem);
  if (e != hipSuccess) return e;
  if (occ < 1) occ = 1;
  *bpc = blocks_per_cu > 0 && blocks_per_cu < occ ? blocks_per_cu : occ;
  return hipSuccess;
}

template <int WAVES, int TG, bool LB, bool EMIT = false>
static hipError_t launch_pruned_lb(const SweepArgs &A, int nmax, int bpc, int n_cu,
                                   hipStream_t st) {
  const size_t shmem = (size_t)WAVES * wave_lds_bytes(nmax, LB, TG, A.S);
  const int64_t need = (A.n_items + WAVES - 1) / WAVES;
  int64_t grid = (int64_t)(bpc > 0 ? bpc : 1) * n_cu;
  if (grid > need) grid = need;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL((sweep_pruned_kernel<WAVES, TG, LB, EMIT>), dim3((unsigned)grid),
                     dim3(WAVES * kWave), shmem, st, A, nmax);
  return hipGetLastError();
}

// Occupancy of WAVES-wave blocks: the LDS-staged bases when they keep the
// occupancy of the register form.
template <int WAVES, int TG>
struct PrunedChoice {
  int bpc = 0;
  bool lds_basis = false;
  hipError_t query(int nmax, int S, int blocks_per_cu) {
    int occ_reg = 0, occ_lds = 0;
    hipError_t e = pruned_occupancy<WAVES, TG, false>(nmax, S, blocks_per_cu, &occ_reg);
    if (e == hipSuccess) e = pruned_occupancy<WAVES, TG, true>(nmax, S, blocks_per_cu, &occ_lds);
    lds_basis = occ_lds >= occ_reg && occ_lds > 0;
    bpc = lds_basis ? occ_lds : occ_reg;
    return e;
  }
  int waves() const { return bpc * WAVES; }
  hipError_t launch(const SweepArgs &A, int nmax, int n_cu, hipStream_t st) const {
    if (bpc < 1) return hipErrorInvalidValue;
    return lds_basis ? launch_pruned_lb<WAVES, TG, true>(A, nmax, bpc, n_cu, st)
                     : launch_pruned_lb<WAVES, TG, false>(A, nmax, bpc, n_cu, st);
  }
};

// waves_per_block 0: the block size with the most resident waves per CU,
// counted up to 6 per SIMD (larger blocks on ties).  A seventh wave per SIMD
// (1-wave blocks at 72 VGPRs) measured slower on the 256-step workload
// (26.5 ms against 22.3 ms at six): the extra waves mostly add L1 pressure.
constexpr int kAutoWavesPerCu = 24;

template <int TG>
static hipError_t launch_pruned_tg(const SweepArgs &A, int nmax, const LaunchPlan &plan,
                                   int n_cu, hipStream_t st) {
  PrunedChoice<4, TG> c4;
  PrunedChoice<2, TG> c2;
  PrunedChoice<1, TG> c1;
  const int w = plan.waves_per_block;
  hipError_t e = hipSuccess;
  if (w == 0 || w == 4) e = c4.query(nmax, A.S, plan.blocks_per_cu);
  if (e == hipSuccess && (w == 0 || w == 2)) e = c2.query(nmax, A.S, plan.blocks_per_cu);
  if (e == hipSuccess && (w == 0 || w == 1)) e = c1.query(nmax, A.S, plan.blocks_per_cu);
  if (e != hipSuccess) return e;
  if (w == 4) return c4.launch(A, nmax, n_cu, st);
  if (w == 2) return c2.launch(A, nmax, n_cu, st);
  if (w == 1) return c1.launch(A, nmax, n_cu, st);
  if (w != 0) return hipErrorInvalidValue;
  const int n4 = min(c4.waves(), kAutoWavesPerCu), n2 = min(c2.waves(), kAutoWavesPerCu),
            n1 = min(c1.waves(), kAutoWavesPerCu);
  if (n4 >= n2 && n4 >= n1) return c4.launch(A, nmax, n_cu, st);
  if (n2 >= n1) return c2.launch(A, nmax, n_cu, st);
  return c1.launch(A, nmax, n_cu, st);
}

hipError_t enqueue_sweep_pruned(const SweepArgs &A, int max_atoms, const LaunchPlan &plan,
                                int n_cu, hipStream_t st) {
  if (A.n_items <= 0) return hipSuccess;
  const int T = (A.S + kWave - 1) / kWave;
  if (!A.emit_x) {
    // grouped classes first (their kernels find their ranges in A.small),
    // the 32-lane ligands in one or (split) two classes
    const int c16 = min(plan.group16_atoms, max_atoms);
    const int c32 = min(plan.group32_atoms, max_atoms);
    const int split = c32 > c16 ? plan.group32_split : 0;
    hipError_t e = hipSuccess;
    if (c16 > 0) e = enqueue_sweep_group(A, 16, 0, (c16 + 15) / 16 * 16, plan, n_cu, st);
    // the 32-lane classes (the same bounds the LPT kernel sorted by), each
    // with the LDS of its largest ligand
    for (int cls = 1, lo = c16; e == hipSuccess && lo < c32; ++cls) {
      const int hi = split > 0 ? min(c32, lo + split) : c32;
      e = enqueue_sweep_group(A, 32, cls, (hi + 15) / 16 * 16, plan, n_cu, st);
      lo = hi;
    }
    if (e != hipSuccess) return e;
    if (max_atoms <= max(c16, c32)) return hipSuccess;  // the last class is empty
  }
  const int nmax = (max_atoms + 15) / 16 * 16;
  if (A.emit_x) {  // profile emission: S == 256 (checked by the caller)
    if (T != 4) return hipErrorInvalidValue;
    int bpc = 0;
    hipError_t e = pruned_occupancy<4, 4, false, true>(nmax, A.S, plan.blocks_per_cu, &bpc);
    if (e != hipSuccess) return e;
    if (bpc < 1) return hipErrorInvalidValue;
    return launch_pruned_lb<4, 4, false, true>(A, nmax, bpc, n_cu, st);
  }
  if (T <= 1) return launch_pruned_tg<1>(A, nmax, plan, n_cu, st);
  if (T <= 2) return launch_pruned_tg<2>(A, nmax, plan, n_cu, st);
  if (T <= 4) return launch_pruned_tg<4>(A, nmax, plan, n_cu, st);
  if (T <= 6) return launch_pruned_tg<6>(A, nmax, plan, n_cu, st);
  return launch_pruned_tg<8>(A, nmax, plan, n_cu, st);
}

}  // namespace dock
