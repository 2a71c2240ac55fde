// Learned angle proposal inside the greedy sweep (phase-synchronous form).
//
// All items of a batch advance one rotamer step at a time so the MLP runs as
// large matrix products over every item's features:
//   begin:  stage the rigid pose, set up the first rotamer, write its 64
//           features and its exact validity mask (bump test of all angles);
//   MLP:    predicted score landscape over 256 bins for every item (bin b
//           holds the steps k whose angle 2 pi k/S lies in
//           [2 pi b/256, 2 pi (b+1)/256): k in [ceil(b S/256), ceil((b+1) S/256)),
//           none, one or several depending on S);
//   step:   nominate the top_k bins by prediction among the bins holding a
//           valid step, score every valid step of those bins (plus angle 0)
//           exactly and keep the best; if the predicted margin (best minus
//           the (top_k+1)-th valid prediction) is below the threshold, score
//           every valid step instead (the plain sweep's step, bit for bit);
//           apply, then set up the next rotamer and write its features and
//           mask.
// Validity is never predicted: it is the same exact bump test as the plain
// sweep, so a chosen angle is always a valid one.
#include <hip/hip_runtime.h>

#include "dock_internal.h"
#include "learned_internal.h"
#include "rotamer_step.h"
#include "sweep_common.h"

namespace dock {

// Compaction capacity of the learned kernels' waves: 8 tiles = 512 steps,
// enough for top_k nominated bins of up to ceil(S/256) steps plus angle 0.
constexpr int kLearnedTiles = 8;

// Orderable 32-bit key of (prediction, -bin) for the nomination rounds.
__device__ __forceinline__ uint32_t nom_key(float y, int k) {
  return (float_order(y) & 0xFFFFFF00u) | (uint32_t)(255 - k);
}

// Rotamer index and step bookkeeping of an item.
struct ItemInfo {
  int l, o, n, R, r0, a0, steps;
};

__device__ __forceinline__ ItemInfo item_info(const LearnedArgs &A, int item) {
  ItemInfo I;
  I.l = item / A.sw.n_orient;
  I.o = item - I.l * A.sw.n_orient;
  I.a0 = A.sw.lig.atom_offset[I.l];
  I.n = A.sw.lig.atom_offset[I.l + 1] - I.a0;
  I.r0 = A.sw.lig.rot_offset[I.l];
  I.R = A.sw.lig.rot_offset[I.l + 1] - I.r0;
  I.steps = I.R * A.sw.passes;
  return I;
}

__device__ __forceinline__ RotState setup_step(const LearnedArgs &A, const WaveLds &W,
                                               const ItemInfo &I, int step, int lane) {
  const int rot = I.r0 + step % I.R;
  const RotTopo T = topo_finish(A.sw.lig, topo_words_load(A.sw.lig, rot, lane), lane);
  return rotamer_setup(W, I.n, T, A.sw.lig.move_atoms, lane);
}

// Features and exact validity (S bits) of the rotamer step just set up.
__device__ __forceinline__ void write_step_inputs(const LearnedArgs &A, const WaveLds &W,
                                                  const RotState &RS, int item, int lane) {
  const GridView G = A.sw.grid;
  A.feat[(size_t)item * 64 + lane] = f32_to_bf16(rotamer_feature(W, RS, G, lane));
  rotamer_bump_mask(W, RS, A.sw.r2, zr_threshold(A.sw.r2 + kPruneMargin), A.sw.S, lane);
  // lane t writes the valid mask of tile t; steps from S on are not angles
  if (lane < A.tiles) {
    const uint64_t bumps = ((uint64_t)W.BM[2 * lane + 1] << 32) | (uint64_t)W.BM[2 * lane];
    const int left = A.sw.S - lane * kWave;
    const uint64_t range = left >= kWave ? ~0ull : ((1ull << left) - 1ull);
    A.valid[(size_t)item * A.tiles + lane] = ~bumps & range;
  }
}

__device__ __forceinline__ void finish_item(const LearnedArgs &A, const WaveLds &W,
                                            const ItemInfo &I, int lane) {
  const float total = pose_total(W, I.n, lane);
  if (lane == 0) {
    if (A.sw.all_scores) A.sw.all_scores[(size_t)I.l * A.sw.n_orient + I.o] = total;
    atomicMax(A.sw.keys + I.l, (unsigned long long)best_key(total, (uint32_t)I.o));
  }
}

__device__ __forceinline__ void save_pose(const LearnedArgs &A, const WaveLds &W, int item,
                                          int n, int lane) {
  float4 *dst = A.pose + (size_t)item * A.nmax;
  for (int i = lane; i < n; i += kWave) dst[i] = W.X[i];
}

__global__ void __launch_bounds__(kWave) learned_begin_kernel(LearnedArgs A) {
  extern __shared__ float4 dyn_lds[];
  const int lane = threadIdx.x;
  const WaveLds W((char *)dyn_lds, A.nmax, false, kLearnedTiles);
  for (int item = blockIdx.x; item < A.sw.n_items; item += gridDim.x) {
    const ItemInfo I = item_info(A, item);
    if (A.sw.status[I.l] != 0) continue;
    stage_pose(W, A.sw.grid, A.sw.lig.xyz + 3 * (size_t)I.a0, I.n,
               A.sw.orient + 12 * ((size_t)I.l * A.sw.orient_stride + I.o), lane);
    if (I.steps == 0) {
      finish_item(A, W, I, lane);
    } else {
      const RotState RS = setup_step(A, W, I, 0, lane);
      write_step_inputs(A, W, RS, item, lane);
      save_pose(A, W, item, I.n, lane);
    }
    wave_lds_sync();
  }
}

// Best key over the valid steps compacted in W.CK[0, nvalid), scored two
// tiles at a time.
__device__ __forceinline__ uint64_t score_compacted_list(const WaveLds &W, const RotState &RS,
                                                         const GridView &G, const GridScaled &GS,
                                                         __amdgpu_buffer_rsrc_t grsrc,
                                                         const float2 *cs, int nvalid, float s0,
                                                         int lane) {
  uint64_t best = 0ull;
  const int tc = (nvalid + kWave - 1) / kWave;
  for (int t0 = 0; t0 < tc; t0 += 2) {
    const uint64_t b =
        tc - t0 >= 2 ? score_compacted<2, false>(W, RS, G, GS, grsrc, cs, nvalid, s0, lane, t0)
                     : score_compacted<1, false>(W, RS, G, GS, grsrc, cs, nvalid, s0, lane, t0);
    best = b > best ? b : best;
  }
  return best;
}

__global__ void __launch_bounds__(kWave) learned_step_kernel(LearnedArgs A, int step) {
  extern __shared__ float4 dyn_lds[];
  const int lane = threadIdx.x;
  const WaveLds W((char *)dyn_lds, A.nmax, false, kLearnedTiles);
  const GridView G = A.sw.grid;
  const GridScaled GS = grid_scaled(G);
  const __amdgpu_buffer_rsrc_t grsrc = grid_rsrc(G);
  const int S = A.sw.S;
  for (int item = blockIdx.x; item < A.sw.n_items; item += gridDim.x) {
    const ItemInfo I = item_info(A, item);
    if (A.sw.status[I.l] != 0 || step >= I.steps) continue;
    const float4 *src = A.pose + (size_t)item * A.nmax;
    for (int i = lane; i < I.n; i += kWave) W.X[i] = src[i];
    wave_lds_sync();
    const RotState RS = setup_step(A, W, I, step, lane);
    const float s0 = rotamer_s0(W, RS, lane);
    const uint64_t *valid = A.valid + (size_t)item * A.tiles;
    // predictions of this item's 256 bins; bins without a valid step are out
    // of the race (lane holds bins lane, 64 + lane, 128 + lane, 192 + lane)
    const float *y = A.pred + (size_t)item * 256;
    uint32_t key[4];
    bool any_valid = false;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int b = t * kWave + lane;
      const int k0 = (b * S + 255) >> 8, cnt = (((b + 1) * S + 255) >> 8) - k0;  // <= 16 steps
      uint64_t bits = 0ull;
      if (cnt > 0) {
        const int wi = k0 >> 6, lo = k0 & 63;
        uint64_t w = valid[wi] >> lo;
        if (lo + cnt > kWave) w |= valid[wi + 1] << (kWave - lo);  // the bin spans two words
        bits = w & ((1ull << cnt) - 1ull);
      }
      key[t] = bits ? nom_key(y[b], b) : 0u;
      any_valid = any_valid || __ballot(bits != 0ull) != 0ull;
    }
    // nomination rounds: the top_k valid bins, then the next one for the margin
    int nom = -1;  // lane j < top_k receives the j-th nominated bin
    uint32_t first = 0u, kth1 = 0u;
    for (int j = 0; j <= A.top_k; ++j) {
      uint32_t mine = key[0];
#pragma unroll
      for (int t = 1; t < 4; ++t) mine = key[t] > mine ? key[t] : mine;
      const uint32_t win = wave_max_u32(mine);
      if (win == 0u) break;
      if (j == 0) first = win;
      if (j == A.top_k) {
        kth1 = win;
        break;
      }
      const int kbin = 255 - (int)(win & 0xFFu);
      if (lane == j) nom = kbin;
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (key[t] == win) key[t] = 0u;
    }
    const float margin = kth1 ? order_float(first | 0xFFu) - order_float(kth1 | 0xFFu) : 3.0e38f;
    const bool fallback = any_valid && margin < A.margin;
    uint64_t best = 0ull;
    if (fallback) {  // the plain step over every valid angle
      for (int t0 = 0; t0 < A.tiles; t0 += 4) {
        uint64_t vm[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) vm[t] = t0 + t < A.tiles ? valid[t0 + t] : 0ull;
        int nvalid;
        const uint64_t key4 =
            best_valid_step<4, false>(W, RS, G, GS, grsrc, A.sw.cs, vm, t0, s0, lane, nvalid);
        best = key4 > best ? key4 : best;
      }
      if (lane == 0) atomicAdd(A.n_fallback + I.l, 1);
    } else if (any_valid) {
      // steps of the nominated bins as an S-bit mask (the bump-mask words are
      // free until the next step's inputs are written)
      for (int i = lane; i < 2 * A.tiles; i += kWave) W.BM[i] = 0u;
      wave_lds_sync();
      if (nom >= 0) {
        const int k1 = ((nom + 1) * S + 255) >> 8;
        for (int k = (nom * S + 255) >> 8; k < k1; ++k) atomicOr(&W.BM[k >> 5], 1u << (k & 31));
      }
      wave_lds_sync();
      // valid steps of the nominated bins, plus angle 0, compacted in order
      int nvalid = 0;
      for (int t = 0; t < A.tiles; ++t) {
        const bool nominated = (W.BM[2 * t + (lane >> 5)] >> (lane & 31)) & 1u;
        const uint64_t m = valid[t] & (__ballot(nominated) | (t == 0 ? 1ull : 0ull));
        if ((m >> lane) & 1ull) W.CK[lanes_before(m, nvalid)] = (int16_t)(t * kWave + lane);
        nvalid += __popcll(m);
      }
      wave_lds_sync();
      best = score_compacted_list(W, RS, G, GS, grsrc, A.sw.cs, nvalid, s0, lane);
      wave_lds_sync();
    }
    best = wave_max_u64(best);
    const int kb = best ? (int)key_index(best) : -1;
    if (lane == 0)
      A.sw.kstar[((size_t)I.r0 * A.sw.n_orient + (size_t)I.o * I.R) * A.sw.passes + step] =
          (int16_t)kb;
    if (kb > 0) {
      const float2 cs = A.sw.cs[kb];
      rotamer_apply(W, RS, G, cs.x, cs.y, lane);
    }
    if (step + 1 < I.steps) {
      const RotState RN = setup_step(A, W, I, step + 1, lane);
      write_step_inputs(A, W, RN, item, lane);
      save_pose(A, W, item, I.n, lane);
    } else {
      finish_item(A, W, I, lane);
    }
    wave_lds_sync();
  }
}

static unsigned grid_for(int n_items, int n_cu) {
  const int64_t g = (int64_t)n_cu * 16;
  return (unsigned)(n_items < g ? (n_items > 0 ? n_items : 1) : g);
}

hipError_t enqueue_learned_begin(const LearnedArgs &A, int n_cu, hipStream_t st) {
  if (A.sw.n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(learned_begin_kernel, dim3(grid_for(A.sw.n_items, n_cu)), dim3(kWave),
                     wave_lds_bytes(A.nmax, false, kLearnedTiles, A.sw.S), st, A);
  return hipGetLastError();
}

hipError_t enqueue_learned_step(const LearnedArgs &A, int step, int n_cu, hipStream_t st) {
  if (A.sw.n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(learned_step_kernel, dim3(grid_for(A.sw.n_items, n_cu)), dim3(kWave),
                     wave_lds_bytes(A.nmax, false, kLearnedTiles, A.sw.S), st, A, step);
  return hipGetLastError();
}

}  // namespace dock
