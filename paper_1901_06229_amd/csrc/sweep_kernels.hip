// Greedy rotamer sweep on gfx950: batch preparation, the persistent
// work-stealing sweep, and the per-ligand finalisation.
//
// Mapping (wave per item).  An item is one (ligand, orientation) restart
// (paper §4.1: restarts are independent and form the outer parallel level).
// Each 64-lane wave of a persistent grid claims items from a global counter
// (work stealing over a cost-sorted list, so ligands of very different size
// balance), stages the ligand in LDS, and walks its rotamers in order
// (fragments are sequential, paper §4.1).  For each rotamer the lanes take
// angle steps: lane k rotates the moving atoms by theta_k, tests every cross
// pair against the bump radius (ballot-driven early exit), sums the voxel
// values, and a wave-wide max over packed (score, -k) keys picks the angle.
// Only the chosen angle is applied to the LDS pose (paper §4.1: rotation and
// scoring are fused so no candidate pose is stored).
#include <hip/hip_runtime.h>

#include "dock_internal.h"
#include "sweep_common.h"

namespace dock {

// ---------------------------------------------------------------- tables
__global__ void cs_table_kernel(float2 *cs, int S) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= S) return;
  const double two_pi = 6.283185307179586476925286766559;
  double th = two_pi * (double)k / (double)S;
  cs[k] = make_float2((float)cos(th), (float)sin(th));
}

// ---------------------------------------------------------------- validation
// One wave per ligand; writes DOCK_OK or an error code into status[l].  The
// ligand's offsets are checked first (wave-uniform); only then do the lanes
// take its rotamers in turn and walk their moving lists, so every read stays
// inside the arrays the checked offsets bound.
constexpr int kValidateWaves = 4;

__global__ void __launch_bounds__(kValidateWaves * kWave)
    validate_kernel(LigView L, int max_atoms, int max_rot, int32_t *status, int32_t *n_bad) {
  const int lane = threadIdx.x & (kWave - 1);
  const int l = blockIdx.x * kValidateWaves + (int)(threadIdx.x / kWave);
  if (l >= L.n_ligands) return;  // whole waves
  int err = 0;
  const int a0 = L.atom_offset[l], a1 = L.atom_offset[l + 1];
  const int r0 = L.rot_offset[l], r1 = L.rot_offset[l + 1];
  const int n = a1 - a0, R = r1 - r0;
  if (a0 < 0 || a1 < a0 || (int64_t)a1 > L.total_atoms || r0 < 0 || r1 < r0 ||
      (int64_t)r1 > L.total_rot)
    err = -1;
  else if (n < 1 || n > max_atoms || R > max_rot)
    err = -2;
  if (!err) {
    bool bad = false;
    for (int r = r0 + lane; r < r1 && !bad; r += kWave) {
      const int a = L.rot_axis[2 * r], b = L.rot_axis[2 * r + 1];
      const int m0 = L.move_offset[r], m1 = L.move_offset[r + 1];
      if (a < 0 || a >= n || b < 0 || b >= n || a == b || m0 < 0 || m1 < m0 ||
          (int64_t)m1 > L.total_move || m1 - m0 > n - 2) {
        bad = true;
        break;
      }
      // the list is read 8 entries at a time (all loads in flight, then the
      // checks in order): the same verdict as one entry at a time, with an
      // eighth of the memory round trips
      int prev = -1;
      for (int t0 = m0; t0 < m1 && !bad; t0 += 8) {
        int e[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) e[q] = t0 + q < m1 ? (int)L.move_atoms[t0 + q] : 0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          if (t0 + q >= m1) break;
          const int i = e[q];
          if (i <= prev || i >= n || i == a || i == b) {
            bad = true;
            break;
          }
          prev = i;
        }
      }
    }
    if (__ballot(bad) != 0ull) err = -1;
  }
  if (lane == 0) {
    status[l] = err;
    if (err) atomicAdd(n_bad, 1);
  }
}

// ---------------------------------------------------------------- LPT order
// Cost of a ligand: sum_r m_r (S + q_r) (per-angle atom work plus pair setup),
// bucketed on a log2 scale; a counting sort emits buckets from the most
// expensive down.  Order inside a bucket is irrelevant to the results.
// Size class c (0: at most c16 atoms; then the 32-lane ligands, at most c32,
// in classes split atoms wide from c16 up, one class when split is 0; the
// rest last) leads the sort key, so every class is a contiguous range of the
// order.  A block counts its ligands per bucket in
// LDS and adds each nonzero count to the global one (one atomic per block
// and bucket instead of one per ligand on a few hundred addresses).
constexpr int kLptThreads = 256;
static_assert(kSortBuckets <= 1024, "one scan thread per bucket");
__global__ void __launch_bounds__(kLptThreads)
    lpt_bucket_kernel(LigView L, int S, const int32_t *status, int c16, int split, int c32,
                      int32_t *bucket_of, int32_t *counts) {
  __shared__ int32_t hist[kSortBuckets];
  for (int i = threadIdx.x; i < kSortBuckets; i += kLptThreads) hist[i] = 0;
  __syncthreads();
  const int l = blockIdx.x * kLptThreads + threadIdx.x;
  if (l < L.n_ligands) {
    float cost = 1.0f;
    int cls = kClasses - 1;
    if (status[l] == 0) {
      int n = L.atom_offset[l + 1] - L.atom_offset[l];
      cls = n <= c16   ? 0
            : n <= c32 ? 1 + (split > 0 ? (n - c16 - 1) / split : 0)
                       : kClasses - 1;
      for (int r = L.rot_offset[l]; r < L.rot_offset[l + 1]; ++r) {
        int m = L.move_offset[r + 1] - L.move_offset[r];
        cost += (float)m * ((float)S + (float)(n - m - 2));
      }
    }
    int b = (int)(log2f(cost) * 2.0f);
    b = b < 0 ? 0 : (b >= kLptBuckets ? kLptBuckets - 1 : b);
    b += cls * kLptBuckets;
    bucket_of[l] = b;
    atomicAdd(&hist[b], 1);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kSortBuckets; i += kLptThreads)
    if (hist[i]) atomicAdd(&counts[i], hist[i]);
}

// Cursors: classes in order, inside a class the most expensive bucket first;
// the class ranges are recorded for the sweep kernels.  One thread per
// bucket (in that order), an exclusive scan in LDS.
__global__ void __launch_bounds__(kSortBuckets)
    lpt_scan_kernel(const int32_t *counts, int32_t *cursor, int32_t *small) {
  __shared__ int32_t s[2][kSortBuckets];
  const int p = threadIdx.x;  // position in the scan order
  const int c = p / kLptBuckets, bucket = c * kLptBuckets + (kLptBuckets - 1 - p % kLptBuckets);
  const int v = counts[bucket];
  int in = 0;
  s[0][p] = v;
  __syncthreads();
  for (int d = 1; d < kSortBuckets; d *= 2) {  // inclusive Hillis-Steele scan
    s[in ^ 1][p] = s[in][p] + (p >= d ? s[in][p - d] : 0);
    in ^= 1;
    __syncthreads();
  }
  const int incl = s[in][p];
  cursor[bucket] = incl - v;
  if (p % kLptBuckets == 0) small[kClassBegin + c] = incl - v;
  if (p % kLptBuckets == kLptBuckets - 1) small[kClassEnd + c] = incl;
}

// Input order: every ligand is in the last class.
__global__ void single_class_kernel(int n_ligands, int32_t *small) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int c = 0; c < kClasses; ++c) {
    small[kClassBegin + c] = c == kClasses - 1 ? 0 : n_ligands;
    small[kClassEnd + c] = n_ligands;
  }
}

// Each ligand's slot in the order: its rank among the block's ligands of its
// bucket (LDS atomics) after the range the block reserves in that bucket
// (one global atomic per block and bucket).  Order inside a bucket does not
// affect any result.
__global__ void __launch_bounds__(kLptThreads)
    lpt_scatter_kernel(int n_ligands, const int32_t *bucket_of, int32_t *cursor,
                       int32_t *order) {
  __shared__ int32_t cnt[kSortBuckets], base[kSortBuckets];
  for (int i = threadIdx.x; i < kSortBuckets; i += kLptThreads) cnt[i] = 0;
  __syncthreads();
  const int l = blockIdx.x * kLptThreads + threadIdx.x;
  int b = 0, rank = 0;
  if (l < n_ligands) {
    b = bucket_of[l];
    rank = atomicAdd(&cnt[b], 1);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kSortBuckets; i += kLptThreads)
    if (cnt[i]) base[i] = atomicAdd(&cursor[i], cnt[i]);
  __syncthreads();
  if (l < n_ligands) order[base[b] + rank] = l;
}

__global__ void fill_i32_kernel(int32_t *p, int n, int32_t v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void identity_order_kernel(int n, int32_t *order) {
  int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l < n) order[l] = l;
}

// Zero the per-call counters and keys (a kernel, not a memset, so the whole
// sequence can be captured in a graph and replayed).
__global__ void reset_kernel(int n_ligands, int32_t *small, int n_small,
                             unsigned long long *keys) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_small) small[i] = 0;
  if (i < n_ligands) keys[i] = 0ull;
}

// ---------------------------------------------------------------- the sweep
template <int MAXN, int WAVES>
__global__ void __launch_bounds__(WAVES *kWave)
    sweep_kernel(SweepArgs A) {
  __shared__ float4 sX[WAVES][MAXN];   // current pose
  __shared__ float4 sQ[WAVES][MAXN];   // compacted static cross set of a rotamer
  __shared__ float sV[WAVES][MAXN];    // voxel value of every atom of the pose
  __shared__ uint8_t sMov[WAVES][MAXN];

  const int wv = threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  float4 *X = sX[wv];
  float4 *Q = sQ[wv];
  float *V = sV[wv];
  uint8_t *mov = sMov[wv];
  const GridView G = A.grid;
  const int O = A.n_orient, S = A.S;
  const uint64_t lanes_below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

  WorkQueue queue(A.queue, A.n_items, A.claim, (int)(gridDim.x * blockDim.x / kWave));
  for (int item; queue.next(lane, item);) {
    const int slot = item / O;
    const int o = item - slot * O;
    const int l = A.order[slot];
    if (A.status[l] != 0) continue;
    const int a0 = A.lig.atom_offset[l];
    const int n = A.lig.atom_offset[l + 1] - a0;
    const int r0 = A.lig.rot_offset[l];
    const int R = A.lig.rot_offset[l + 1] - r0;
    const float *T = A.orient + 12 * ((size_t)l * A.orient_stride + o);

    for (int i = lane; i < n; i += kWave) {
      const float *p = A.lig.xyz + 3 * (size_t)(a0 + i);
      float3 x = orient_point(T, p[0], p[1], p[2]);
      X[i] = make_float4(x.x, x.y, x.z, 0.0f);
      V[i] = voxel_value(G, x.x, x.y, x.z);
    }
    wave_lds_sync();

    int16_t *kout = A.kstar + ((size_t)r0 * O + (size_t)o * R) * A.passes;
    int step = 0;
    for (int pass = 0; pass < A.passes; ++pass) {
      for (int r = 0; r < R; ++r, ++step) {
        const int ra = A.lig.rot_axis[2 * (r0 + r)];
        const int rb = A.lig.rot_axis[2 * (r0 + r) + 1];
        const int ms = A.lig.move_offset[r0 + r];
        const int m = A.lig.move_offset[r0 + r + 1] - ms;
        const int16_t *mlist = A.lig.move_atoms + ms;
        for (int i = lane; i < n; i += kWave) mov[i] = 0;
        wave_lds_sync();
        for (int t = lane; t < m; t += kWave) mov[mlist[t]] = 1;
        wave_lds_sync();
        // compact the static cross set Q_r (ascending atom order)
        int q = 0;
        for (int base = 0; base < n; base += kWave) {
          int i = base + lane;
          bool st = i < n && !mov[i] && i != ra && i != rb;
          uint64_t mask = __ballot(st);
          if (st) Q[q + __popcll(mask & lanes_below)] = X[i];
          q += __popcll(mask);
        }
        // score of everything that does not move, in atom order
        float cst = 0.0f;
        for (int i = 0; i < n; ++i)
          if (!mov[i]) cst += V[i];
        wave_lds_sync();
        const float4 xa = X[ra];
        const float3 u = bond_axis(xa, X[rb]);

        uint64_t best = 0ull;
        for (int base = 0; base < S; base += kWave) {
          const int k = base + lane;
          const bool active = k < S;
          const float2 cs = A.cs[active ? k : 0];
          bool bump = !active;
          float score = cst;
          for (int t = 0; t < m; ++t) {
            const float4 xi = X[mlist[t]];
            float3 y = rodrigues(xi, xa, u, cs.x, cs.y);
            if (k == 0) y = make_float3(xi.x, xi.y, xi.z);
            if (__ballot(!bump) == 0ull) break;  // every angle of the tile rejected
            for (int j = 0; j < q; ++j) {
              const float4 xj = Q[j];
              float dx = y.x - xj.x, dy = y.y - xj.y, dz = y.z - xj.z;
              float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
              bump = bump || (d2 < A.r2);
            }
            score += voxel_value(G, y.x, y.y, y.z);
          }
          uint64_t key = bump ? 0ull : best_key(score, (uint32_t)k);
          best = key > best ? key : best;
        }
        best = wave_max_u64(best);
        const int kb = best ? (int)key_index(best) : -1;
        if (lane == 0) kout[step] = (int16_t)kb;
        if (kb > 0) {
          const float2 cs = A.cs[kb];
          for (int t = lane; t < m; t += kWave) {
            const int i = mlist[t];
            float3 y = rodrigues(X[i], xa, u, cs.x, cs.y);
            X[i] = make_float4(y.x, y.y, y.z, 0.0f);
            V[i] = voxel_value(G, y.x, y.y, y.z);
          }
        }
        wave_lds_sync();
      }
    }
    float total = 0.0f;
    for (int i = 0; i < n; ++i) total += V[i];
    if (lane == 0) {
      if (A.all_scores) A.all_scores[(size_t)l * O + o] = total;
      atomicMax(A.keys + l, (unsigned long long)best_key(total, (uint32_t)o));
    }
    wave_lds_sync();
  }
}

// ---------------------------------------------------------------- finalise
// One wave per ligand: decode the winning orientation, replay its recorded
// angle choices with the sweep's own arithmetic, write the pose.
template <int MAXN, int MODE>
__global__ void __launch_bounds__(kWave) finalize_kernel(SweepArgs A, FinalOut F) {
  __shared__ float4 X[MAXN];
  const int l = blockIdx.x;
  const int lane = threadIdx.x;
  if (l >= A.lig.n_ligands) return;
  const uint64_t key = A.keys[l];
  const int O = A.n_orient;
  const int a0 = A.lig.atom_offset[l];
  const int r0 = A.lig.rot_offset[l];
  if (A.status[l] != 0 || key == 0ull) {
    if (lane == 0) {
      F.best_orient[l] = -1;
      F.best_score[l] = __int_as_float(0x7fc00000);
      if (F.align_idx) F.align_idx[l] = -1;
    }
    return;
  }
  const int n = A.lig.atom_offset[l + 1] - a0;
  const int R = A.lig.rot_offset[l + 1] - r0;
  const int o = (int)key_index(key);
  const float *T = A.orient + 12 * ((size_t)l * A.orient_stride + o);
  for (int i = lane; i < n; i += kWave) {
    const float *p = A.lig.xyz + 3 * (size_t)(a0 + i);
    float3 x = orient_point(T, p[0], p[1], p[2]);
    X[i] = make_float4(x.x, x.y, x.z, 0.0f);
  }
  wave_lds_sync();
  const int16_t *ks = A.kstar + ((size_t)r0 * O + (size_t)o * R) * A.passes;
  // The replay is serial in the steps, so each step's inputs (choice, axis
  // atoms, moving-list range, cos/sin) are loaded up front, 64 steps at a
  // time with one step per lane, and taken from the owning lane in the loop:
  // no step waits on a chain of global loads.
  const int steps = R * A.passes;
  for (int c0 = 0; c0 < steps; c0 += kWave) {
    int k = -1, ra = 0, rb = 0, ms = 0, m = 0;
    float cx = 1.0f, sy = 0.0f;
    if (c0 + lane < steps) {
      const int s = c0 + lane, r = s % R;
      k = ks[s];
      F.angle_idx[(size_t)r0 * A.passes + s] = (int16_t)k;
      if (k > 0) {
        ra = A.lig.rot_axis[2 * (r0 + r)];
        rb = A.lig.rot_axis[2 * (r0 + r) + 1];
        ms = A.lig.move_offset[r0 + r];
        m = A.lig.move_offset[r0 + r + 1] - ms;
        const float2 cs = A.cs[k];
        cx = cs.x;
        sy = cs.y;
      }
    }
    const int cnt = min(kWave, steps - c0);
    for (int j = 0; j < cnt; ++j) {
      if (__builtin_amdgcn_readlane(k, j) <= 0) continue;  // wave-uniform
      const int sra = __builtin_amdgcn_readlane(ra, j), srb = __builtin_amdgcn_readlane(rb, j);
      const int sms = __builtin_amdgcn_readlane(ms, j), sm = __builtin_amdgcn_readlane(m, j);
      const float scx = lane_bcast(cx, j), ssy = lane_bcast(sy, j);
      const float4 xa = X[sra];
      const float3 u = bond_axis(xa, X[srb]);
      wave_lds_sync();
      for (int t = lane; t < sm; t += kWave) {
        const int i = A.lig.move_atoms[sms + t];
        float3 y;
        if (MODE == kSweepPruned) {
          const Cyl c = cyl_of(X[i], xa, u);
          y = rot_apply(rot_basis(c, xa, u), scx, ssy);
        } else {
          y = rodrigues(X[i], xa, u, scx, ssy);
        }
        X[i] = make_float4(y.x, y.y, y.z, 0.0f);
      }
      wave_lds_sync();
    }
  }
  for (int i = lane; i < n; i += kWave) {
    float *q = F.xyz_out + 3 * (size_t)(a0 + i);
    q[0] = X[i].x;
    q[1] = X[i].y;
    q[2] = X[i].z;
  }
  if (lane == 0) {
    F.best_orient[l] = o;
    F.best_score[l] = key_score(key);
    if (F.align_idx) F.align_idx[l] = F.item_align ? F.item_align[(size_t)l * O + o] : (int16_t)-1;
  }
}

// ---------------------------------------------------------------- launches
static inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

hipError_t enqueue_fill_i32(int32_t *p, int n, int32_t v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_i32_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t enqueue_prepare(const SweepArgs &A, int max_atoms, int max_rot, bool lpt, int c16,
                           int split, int c32, int32_t *bucket_of, int32_t *counts,
                           int32_t *cursor, int32_t *n_bad, hipStream_t st) {
  const int L = A.lig.n_ligands;
  const int nsmall = kSmallInts;
  int n_reset = L > nsmall ? L : nsmall;
  hipLaunchKernelGGL(reset_kernel, dim3(blocks_for(n_reset, 256)), dim3(256), 0, st, L,
                     A.small, nsmall, A.keys);
  hipLaunchKernelGGL(cs_table_kernel, dim3(blocks_for(A.S, 256)), dim3(256), 0, st,
                     const_cast<float2 *>(A.cs), A.S);
  if (L > 0) {
    hipLaunchKernelGGL(validate_kernel, dim3(blocks_for(L, kValidateWaves)), dim3(kValidateWaves * kWave),
                       0, st, A.lig, max_atoms, max_rot, const_cast<int32_t *>(A.status), n_bad);
    if (lpt) {
      hipLaunchKernelGGL(lpt_bucket_kernel, dim3(blocks_for(L, kLptThreads)), dim3(kLptThreads),
                         0, st, A.lig, A.S, A.status, c16, split, c32, bucket_of, counts);
      hipLaunchKernelGGL(lpt_scan_kernel, dim3(1), dim3(kSortBuckets), 0, st, counts, cursor,
                         A.small);
      hipLaunchKernelGGL(lpt_scatter_kernel, dim3(blocks_for(L, kLptThreads)), dim3(kLptThreads),
                         0, st, L, bucket_of, cursor, const_cast<int32_t *>(A.order));
    } else {
      hipLaunchKernelGGL(identity_order_kernel, dim3(blocks_for(L, 256)), dim3(256), 0, st,
                         L, const_cast<int32_t *>(A.order));
      hipLaunchKernelGGL(single_class_kernel, dim3(1), dim3(64), 0, st, L, A.small);
    }
  }
  return hipGetLastError();
}

template <int MAXN, int WAVES>
static hipError_t launch_sweep_t(const SweepArgs &A, int blocks_per_cu, int n_cu,
                                 hipStream_t st) {
  int occ = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &occ, sweep_kernel<MAXN, WAVES>, WAVES * kWave, 0);
  if (e != hipSuccess) return e;
  if (occ < 1) occ = 1;
  int bpc = blocks_per_cu > 0 && blocks_per_cu < occ ? blocks_per_cu : occ;
  int64_t need = (A.n_items + WAVES - 1) / WAVES;
  int64_t grid = (int64_t)bpc * n_cu;
  if (grid > need) grid = need;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL((sweep_kernel<MAXN, WAVES>), dim3((unsigned)grid),
                     dim3(WAVES * kWave), 0, st, A);
  return hipGetLastError();
}

hipError_t enqueue_sweep(const SweepArgs &A, int maxn, const LaunchPlan &plan, int n_cu,
                         hipStream_t st) {
  if (A.n_items <= 0) return hipSuccess;
  const int waves = plan.waves_per_block == 0 ? 4 : plan.waves_per_block;  // 0: automatic
#define DOCK_SWEEP_CASE(N, W)                                                       \
  if (maxn <= N && waves == W)                                                        \
    return launch_sweep_t<N, W>(A, plan.blocks_per_cu, n_cu, st);
  DOCK_SWEEP_CASE(64, 1)
  DOCK_SWEEP_CASE(64, 2)
  DOCK_SWEEP_CASE(64, 4)
  DOCK_SWEEP_CASE(128, 1)
  DOCK_SWEEP_CASE(128, 2)
  DOCK_SWEEP_CASE(128, 4)
  DOCK_SWEEP_CASE(256, 1)
  DOCK_SWEEP_CASE(256, 2)
  DOCK_SWEEP_CASE(256, 4)
#undef DOCK_SWEEP_CASE
  return hipErrorInvalidValue;
}

hipError_t enqueue_finalize(const SweepArgs &A, const FinalOut &F, int maxn, SweepMode mode,
                            hipStream_t st) {
  const int L = A.lig.n_ligands;
  if (L <= 0) return hipSuccess;
#define DOCK_FIN(N, M) \
  hipLaunchKernelGGL((finalize_kernel<N, M>), dim3(L), dim3(kWave), 0, st, A, F)
  if (mode == kSweepPruned) {
    if (maxn <= 64) DOCK_FIN(64, kSweepPruned);
    else if (maxn <= 128) DOCK_FIN(128, kSweepPruned);
    else DOCK_FIN(256, kSweepPruned);
  } else {
    if (maxn <= 64) DOCK_FIN(64, kSweepDirect);
    else if (maxn <= 128) DOCK_FIN(128, kSweepDirect);
    else DOCK_FIN(256, kSweepDirect);
  }
#undef DOCK_FIN
  return hipGetLastError();
}

}  // namespace dock
