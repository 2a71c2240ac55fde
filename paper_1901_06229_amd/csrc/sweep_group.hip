// Grouped mapping of the pruned sweep for small ligands: a wave docks 64 / G
// orientations of one ligand at once, one G-lane group per (ligand,
// orientation) item (G = 16 or 32).
//
// Why: a rotamer step of a small ligand leaves most of a 64-lane wave idle
// in its per-step work -- the clash arcs of ~14 kept pairs, the application
// of the chosen angle to ~7 moving atoms, the reductions, a partly filled
// score tile.  The items of one ligand share its topology (atom count,
// rotamers, moving and static lists), so groups of one wave run the same
// loops in lockstep and only their data differ: each group keeps its own
// pose, bump bits and compacted steps; the moving / static lists and the
// kept-pair list (pairs tagged with their group) are shared by the wave.
// Per item, that divides the per-step work by the number of groups where it
// fits in G lanes.
//
// Every result is bitwise the one-item-per-wave kernel's: the same functions
// place atoms, test and arc pairs, index voxels and key angles; scores add
// the moving atoms in list order onto the static score, and the static and
// final scores use the mapping-independent chunked atom sum.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "dock_internal.h"
#include "sweep_common.h"
#include "rotamer_step.h"

namespace dock {

// Ring of compacted steps per group (entries), steps compacted per append
// (the chunk), kept-pair list of the wave (entries).
template <int G> constexpr int kGroupRing = 4 * G;
template <int G> constexpr int kGroupChunk = 2 * G;
constexpr int kGroupScoreTiles = 2;  // compacted G-step tiles scored per full pass
constexpr int kWavePairCap = 384;
// moving atoms whose voxel-unit bases a group holds at once (half its lanes:
// LDS is what bounds the resident waves)
template <int G> constexpr int kGroupBasisAtoms = G / 2;
static_assert(kGroupChunk<16> + kGroupScoreTiles * 16 <= kGroupRing<16>, "ring too small");
static_assert(kGroupChunk<32> + kGroupScoreTiles * 32 <= kGroupRing<32>, "ring too small");

__host__ __device__ inline int round16(int b) { return (b + 15) / 16 * 16; }

// LDS of one wave.  LDS bounds how many waves a compute unit holds, and these
// kernels run faster with every wave added (latency-bound), so it is kept
// small.
//   shared:  Q, M (uint8 [nmax]) static and moving lists of the step,
//            slot (uint8 [nmax]) an atom's entry in ZRc: moving atom t -> t,
//            static atom Q[p] -> m + p, axis atoms kNoSlot (ligands of the
//            grouped classes have at most 192 atoms),
//            U (float4 [NG]) each group's unit bond axis (its axis point is
//            the pose's atom ra)
//   scratch: one block per group, contiguous: the moving atoms' voxel-unit
//            bases (float [9][G / 2]) and the ring of compacted steps (int16
//            [4G]) while scoring; the moving atoms' values for the step-0
//            score; during the bump test all of it is the wave's kept-pair
//            list (int [kWavePairCap])
//   groups:  X (float4 [nmax]) pose, x y z and voxel value
//            ZRc (uint32 [nmax]) axial coordinate and |r| about the bond axis,
//            packed for the pair bound (pack_zr), of the moving atoms (in
//            list order), then of the static ones
//            BM (uint32 [(S + 31) / 32]) bump bits
constexpr uint8_t kNoSlot = 0xFF;  // above every moving-list position
static_assert(kGroupMaxAtoms16 < kNoSlot && kGroupMaxAtoms32 < kNoSlot, "uint8 atom lists");
template <int G>
__host__ __device__ inline int group_shared_bytes(int nmax) {
  return round16(nmax * 3) + (kWave / G) * 16;
}
template <int G>
__host__ __device__ constexpr int group_scratch_bytes() {
  return (9 * kGroupBasisAtoms<G> * 4 + kGroupRing<G> * 2 + 15) / 16 * 16;
}
static_assert(group_scratch_bytes<16>() >= 4 * kGroupMaxAtoms16, "scratch too small");
static_assert(group_scratch_bytes<32>() >= 4 * kGroupMaxAtoms32, "scratch too small");
static_assert((kWave / 16) * group_scratch_bytes<16>() >= 4 * kWavePairCap, "pair list");
static_assert((kWave / 32) * group_scratch_bytes<32>() >= 4 * kWavePairCap, "pair list");
template <int G>
__host__ __device__ inline int group_region_bytes(int nmax, int S) {
  return nmax * 16 + nmax * 4 + round16(4 * ((S + 31) / 32));
}
template <int G>
__host__ __device__ inline int group_wave_bytes(int nmax, int S) {
  return group_shared_bytes<G>(nmax) +
         (kWave / G) * (group_scratch_bytes<G>() + group_region_bytes<G>(nmax, S));
}

template <int G>
struct GroupLds {
  uint8_t *Q, *M, *slot;
  float4 *U;      // [NG]
  int *PL;        // the wave's kept-pair list
  char *regions;  // group 0's region; group g's at + g * region
  int region;
  int nmax;
  // this group's
  float4 *X;
  uint32_t *ZRc;
  float *B;
  int16_t *CK;
  uint32_t *BM;
  __device__ GroupLds(char *wave_base, int nmax_, int S, int gid) {
    nmax = nmax_;
    Q = (uint8_t *)wave_base;
    M = Q + nmax;
    slot = M + nmax;
    U = (float4 *)(wave_base + round16(nmax * 3));
    char *scr0 = wave_base + group_shared_bytes<G>(nmax);
    PL = (int *)scr0;
    char *scr = scr0 + gid * group_scratch_bytes<G>();
    B = (float *)scr;
    CK = (int16_t *)(scr + 9 * kGroupBasisAtoms<G> * 4);
    regions = scr0 + (kWave / G) * group_scratch_bytes<G>();
    region = group_region_bytes<G>(nmax, S);
    X = group_X(gid);
    ZRc = (uint32_t *)(X + nmax);
    BM = group_BM(gid);
  }
  __device__ __forceinline__ float4 *group_X(int g) const {
    return (float4 *)(regions + g * region);
  }
  __device__ __forceinline__ uint32_t *group_BM(int g) const {
    return (uint32_t *)(regions + g * region + nmax * 20);
  }
};

// Lane bookkeeping of a G-lane group.
template <int G>
struct Grp {
  static constexpr int NG = kWave / G;
  static constexpr uint32_t kLow = G == 32 ? 0xFFFFFFFFu : ((1u << G) - 1u);
  int gid, gl, gbase;
  uint32_t below;  // group lanes below this one
  __device__ explicit Grp(int lane)
      : gid(lane / G), gl(lane % G), gbase(lane / G * G), below((1u << (lane % G)) - 1u) {}
  // this group's bits of a wave ballot (bit i: group lane i)
  __device__ __forceinline__ uint32_t bits(uint64_t ballot) const {
    return (uint32_t)(ballot >> gbase) & kLow;
  }
};

// Sum over each group's lanes in the chunked order (see chunk_sum_wave):
// the group's 16-lane rows are its chunks, added in row order.  acc and the
// result are the same in all lanes of a group.
template <int G>
__device__ __forceinline__ float chunk_sum_group(float acc, float v, int base, int n, int gl) {
  const float rs = row_sum16(v);
  if constexpr (G == 16) {
    return acc + rs;  // one chunk, below n whenever the loop runs
  } else {
    // the other row's sum (rows 2g and 2g + 1 swap: bitmask swizzle, xor 16)
    const float other = __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(rs), 0x401F));
    const bool lo = gl < 16;
    acc += lo ? rs : other;
    if (base + 16 < n) acc += lo ? other : rs;
    return acc;
  }
}

// Maximum of a 32-bit value over each group (all of its lanes get it).
template <int G>
__device__ __forceinline__ uint32_t group_max_u32(uint32_t v) {
  auto mx = [](uint32_t a, uint32_t b) { return a > b ? a : b; };
  v = mx(v, dpp_move<0xB1, 0xF>(0u, v));
  v = mx(v, dpp_move<0x4E, 0xF>(0u, v));
  v = mx(v, dpp_move<0x141, 0xF>(0u, v));
  v = mx(v, dpp_move<0x140, 0xF>(0u, v));
  if constexpr (G == 32) v = mx(v, (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x401F));
  return v;
}

template <int G>
__device__ __forceinline__ uint64_t group_max_u64(uint64_t v) {
  const uint32_t hi = group_max_u32<G>((uint32_t)(v >> 32));
  const uint32_t lo = group_max_u32<G>((uint32_t)(v >> 32) == hi ? (uint32_t)v : 0u);
  return ((uint64_t)hi << 32) | lo;
}

// Voxel-unit rotation bases of moving atoms c0 .. c0 + GB - 1 into the
// group's B (one atom per lane of the group's first GB lanes).
template <int G>
__device__ __forceinline__ void group_bases(const GroupLds<G> &W, const Grp<G> &g, int m, int c0,
                                            float4 xa, float3 u, const GridView &GV) {
  constexpr int GB = kGroupBasisAtoms<G>;
  if (g.gl < GB && c0 + g.gl < m) {
    const Cyl c = cyl_of(W.X[W.M[c0 + g.gl]], xa, u);
    const VoxBasis vb = voxel_basis(rot_basis(c, xa, u), GV);
    float *B = W.B + g.gl;
    B[0 * GB] = vb.px, B[1 * GB] = vb.py, B[2 * GB] = vb.pz;
    B[3 * GB] = vb.ex, B[4 * GB] = vb.ey, B[5 * GB] = vb.ez;
    B[6 * GB] = vb.fx, B[7 * GB] = vb.fy, B[8 * GB] = vb.fz;
  }
}

// Scores of the lane's TC compacted steps kk (-1: none) -- static score plus
// the moving atoms' values in list order, as rotamer_scores computes them.
// cached: m <= GB and B already holds the bases (written once per rotamer
// step and kept across its passes).
template <int G, int TC>
__device__ __forceinline__ void group_scores(const GroupLds<G> &W, const Grp<G> &g, int m,
                                             bool cached, float cst, float4 xa, float3 u,
                                             const GridView &GV, const GridScaled &GS,
                                             __amdgpu_buffer_rsrc_t grsrc,
                                             const float (&cc)[TC], const float (&ss)[TC],
                                             float (&score)[TC]) {
#pragma unroll
  for (int t = 0; t < TC; ++t) score[t] = cst;
  constexpr int GB = kGroupBasisAtoms<G>;
  for (int c0 = 0; c0 < m; c0 += GB) {
    if (!cached) {
      group_bases<G>(W, g, m, c0, xa, u, GV);
      wave_lds_sync();
    }
    const int cnt = min(GB, m - c0);
    auto gather = [&](int tt, float(&v)[TC]) {
      const float *B = W.B + tt;  // group-uniform address: broadcast reads
      const VoxBasis vb{B[0 * GB], B[1 * GB], B[2 * GB], B[3 * GB], B[4 * GB],
                        B[5 * GB], B[6 * GB], B[7 * GB], B[8 * GB]};
      uint32_t off[TC];
#pragma unroll
      for (int t = 0; t < TC; ++t) off[t] = basis_voxel_offset(GS, vb, cc[t], ss[t]);
#pragma unroll
      for (int t = 0; t < TC; ++t) v[t] = grid_load(grsrc, off[t]);
      __builtin_amdgcn_sched_barrier(0);
    };
    auto accumulate = [&](const float(&v)[TC]) {
#pragma unroll
      for (int t = 0; t < TC; ++t) score[t] += v[t];
    };
    float va[TC], vb[TC];
    gather(0, va);
    int tt = 1;
    for (; tt + 1 < cnt; tt += 2) {
      gather(tt, vb);
      accumulate(va);
      gather(tt + 1, va);
      accumulate(vb);
    }
    if (tt < cnt) {
      gather(tt, vb);
      accumulate(va);
      accumulate(vb);
    } else {
      accumulate(va);
    }
    wave_lds_sync();
  }
}

// 1-wave blocks are held to 80 VGPRs (6 waves per SIMD; they fit without
// spills): where LDS allows more than 20 waves per compute unit (the 32-lane
// class, the 16-lane class up to 64 atoms) the launch then picks them.
template <int G, int WAVES>
__global__ void __launch_bounds__(WAVES *kWave) __attribute__((amdgpu_waves_per_eu(WAVES == 1 ? 6 : 1)))
    sweep_group_kernel(SweepArgs args, int nmax, int cls) {
  (void)args;
  const SweepArgs &A = *(const SweepArgs *)__builtin_amdgcn_kernarg_segment_ptr();
  constexpr int NG = kWave / G;
  extern __shared__ float4 dyn_lds[];
  const int wv = threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  const Grp<G> g(lane);
  const int S = A.S;
  const GroupLds<G> W((char *)dyn_lds + (size_t)wv * group_wave_bytes<G>(nmax, S), nmax, S, g.gid);
  const GridView GV = A.grid;
  const GridScaled GS = grid_scaled(GV);
  const __amdgpu_buffer_rsrc_t grsrc = grid_rsrc(GV);
  const int O = A.n_orient;
  const float r2 = A.r2;
  const int thr_q = zr_threshold(r2 + kPruneMargin);
  const float steps_per_rad = (float)S * 0.15915494309189535f;  // S / (2 pi)
  const int words = (S + 31) / 32;
  // bits of a 32-bit bump word below this lane's step, per G-step half
  uint32_t below_bit[32 / G];
#pragma unroll
  for (int h = 0; h < 32 / G; ++h) below_bit[h] = (1u << (h * G + g.gl)) - 1u;
  uint64_t kept_pairs = 0;  // the wave's work counters: kept pairs (wave-uniform),
  uint64_t evals = 0;       // evaluations of this group

  const int cb = A.small[kClassBegin + cls], ce = A.small[kClassEnd + cls];
  const int upl = (O + NG - 1) / NG;  // units (NG orientations) per ligand
  WorkQueue queue(A.small + kClassQueue + cls, (ce - cb) * upl, A.claim, (int)gridDim.x * WAVES);
  for (int unit; queue.next(lane, unit);) {
    const int slot = cb + unit / upl;
    const int o_first = (unit - (slot - cb) * upl) * NG;
    const int o_mine = o_first + g.gid;
    const bool active = o_mine < O;
    const int o = active ? o_mine : o_first;  // an idle group repeats the first one's item
    const int l = A.order[slot];
    if (A.status[l] != 0) continue;
    const int a0 = A.lig.atom_offset[l];
    const int n = A.lig.atom_offset[l + 1] - a0;
    const int r0 = A.lig.rot_offset[l];
    const int R = A.lig.rot_offset[l + 1] - r0;
    {
      const float *T = A.orient + 12 * ((size_t)l * A.orient_stride + o);
      const float *xyz = A.lig.xyz + 3 * (size_t)a0;
      for (int i = g.gl; i < n; i += G) {
        const float3 x = orient_point(T, xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]);
        W.X[i] = make_float4(x.x, x.y, x.z, voxel_value(GV, x.x, x.y, x.z));
      }
    }
    wave_lds_sync();
    int16_t *kout = A.kstar + ((size_t)r0 * O + (size_t)o * R) * A.passes;
    const int steps = R * A.passes;
    int kreg = -1;  // group lane s holds the choice of step s (mod G) until written out
    int step = 0;
    for (int pass = 0; pass < A.passes; ++pass) {
      for (int r = 0; r < R; ++r, ++step) {
        const int rot = r0 + r;
        const int ra = A.lig.rot_axis[2 * rot], rb = A.lig.rot_axis[2 * rot + 1];
        const int ms = A.lig.move_offset[rot];
        const int m = A.lig.move_offset[rot + 1] - ms;
        // moving list, static list and slots: once per wave (shared topology)
        for (int i = lane; i < n; i += kWave) W.slot[i] = kNoSlot;
        wave_lds_sync();
        for (int t = lane; t < m; t += kWave) {
          const int i = A.lig.move_atoms[ms + t];
          W.slot[i] = (uint8_t)t;
          W.M[t] = (uint8_t)i;
        }
        wave_lds_sync();
        int q = 0;
        for (int base = 0; base < n; base += kWave) {
          const int i = base + lane;
          const bool st = i < n && W.slot[i] == kNoSlot && i != ra && i != rb;
          const uint64_t mask = wave_ballot(st);
          if (st) {
            const int pos = lanes_before(mask, q);
            W.Q[pos] = (uint8_t)i;
            W.slot[i] = (uint8_t)(m + pos);
          }
          q += __popcll(mask);
        }
        wave_lds_sync();
        // per group: axis, (z, |r|) of the moving and static atoms, static score
        const float4 xa = W.X[ra];
        const float3 u = bond_axis(xa, W.X[rb]);
        float cst = 0.0f;
        for (int base = 0; base < n; base += G) {
          const int i = base + g.gl;
          float v = 0.0f;
          if (i < n) {
            const float4 xi = W.X[i];
            const int sl = W.slot[i];
            if (sl != kNoSlot) {
              const Cyl c = cyl_of(xi, xa, u);
              W.ZRc[sl] = pack_zr(c.z, cyl_radius(make_float4(c.rx, c.ry, c.rz, c.z)));
            }
            if (sl >= m) v = xi.w;  // everything that does not move (kNoSlot too)
          }
          cst = chunk_sum_group<G>(cst, v, base, n, g.gl);
        }
        for (int w = g.gl; w < words; w += G) W.BM[w] = 0u;
        // the moving atoms' current values, in list order, into the scratch
        // (free until the pair list fills it): read in parallel, added below
        float *mval = W.B;
        for (int t = g.gl; t < m; t += G) mval[t] = W.X[W.M[t]].w;
        wave_lds_sync();
        // the current pose's score (step 0): static score, then the moving
        // atoms' values in list order (independent broadcast reads)
        float s0 = cst;
#pragma unroll 4
        for (int t = 0; t < m; ++t) s0 += mval[t];
        wave_lds_sync();

        // bump bits: pairs whose cylinder bound does not clear r_bump go into
        // the wave's pair list (packed group << 16 | moving-list position << 8
        // | j); their clash arcs are then marked 64 pairs at a time, each
        // lane into its pair's group (that group's axis point is its atom ra,
        // its unit axis is in U)
        if (g.gl == 0) W.U[g.gid] = make_float4(u.x, u.y, u.z, 0.0f);
        int np = 0;  // pairs in the list (wave-uniform)
        auto flush = [&]() {
          wave_lds_sync();
          for (int e0 = 0; e0 < np; e0 += kWave) {
            const int e = e0 + lane;
            bool counted = false;
            if (e < np) {
              const int pk = W.PL[e];
              const int pg = pk >> 16, i = W.M[(pk >> 8) & 0xFF], j = pk & 0xFF;
              const float4 *Xg = W.group_X(pg);
              const float4 pxa = Xg[ra], pu4 = W.U[pg];
              const float3 pu = make_float3(pu4.x, pu4.y, pu4.z);
              const Cyl ci = cyl_of(Xg[i], pxa, pu), cj = cyl_of(Xg[j], pxa, pu);
              mark_pair_arc(W.group_BM(pg), make_float4(ci.rx, ci.ry, ci.rz, ci.z),
                            make_float4(cj.rx, cj.ry, cj.rz, cj.z), pu, r2, S, steps_per_rad);
              counted = o_first + pg < O;  // pairs of idle groups are not work
            }
            kept_pairs += (uint64_t)__popcll(wave_ballot(counted));
          }
          np = 0;
          wave_lds_sync();
        };
        for (int jb = 0; jb < q; jb += G) {
          const bool jin = jb + g.gl < q;
          const int j = jin ? W.Q[jb + g.gl] : 0;
          const uint32_t zrj = W.ZRc[jin ? m + jb + g.gl : 0];
          const int tj = jin ? thr_q : -1;  // lanes past the list keep nothing
          const int pj = (g.gid << 16) | j;
          auto test = [&](const uint32_t mz, int t) {
            const int lb = zr_bound(mz, zrj);
            const uint64_t keep = wave_ballot(lb <= tj);
            if (lb <= tj) W.PL[lanes_before(keep, np)] = pj | (t << 8);
            np += __popcll(keep);
          };
          int t = 0;
          for (; t + 1 < m; t += 2) {  // two moving atoms per turn, both reads first
            const uint32_t mz0 = W.ZRc[t], mz1 = W.ZRc[t + 1];  // group-uniform: broadcasts
            test(mz0, t);
            test(mz1, t + 1);
            if (np > kWavePairCap - 2 * kWave) flush();
          }
          if (t < m) {
            test(W.ZRc[t], t);
            if (np > kWavePairCap - 2 * kWave) flush();
          }
        }
        flush();

        // non-bumping steps: compacted 2G steps at a time into a ring of 4G
        // entries per group and scored in passes of kGroupScoreTiles x G
        // entries as soon as one group has that many unread, so passes stay
        // full across chunks; what is left at the end (< 2G entries) takes
        // one pass of one or two tiles.  Passes run wave-wide; each group
        // reads its own next entries.  Unread entries stay below 2G after a
        // pass and below 4G after an append, so the ring never overwrites them.
        // a step whose moving atoms fit the group's basis slots computes their bases once
        // (the pair list, which shared this scratch, is done)
        const bool cached = m <= kGroupBasisAtoms<G>;
        if (cached) group_bases<G>(W, g, m, 0, xa, u, GV);
        uint64_t best = 0ull;
        int nv = 0;       // entries this group has appended (same in its lanes)
        int rd = 0;       // entries this group has scored
        auto pass = [&](auto tiles) {
          constexpr int TC = decltype(tiles)::value;
          float cc[TC], ss[TC], score[TC];
          int kk[TC];
#pragma unroll
          for (int t = 0; t < TC; ++t) {
            const int jj = rd + t * G + g.gl;
            kk[t] = jj < nv ? W.CK[jj & (kGroupRing<G> - 1)] : -1;
            const float2 cs = A.cs[kk[t] > 0 ? kk[t] : 0];
            cc[t] = cs.x;
            ss[t] = cs.y;
          }
          group_scores<G, TC>(W, g, m, cached, cst, xa, u, GV, GS, grsrc, cc, ss, score);
#pragma unroll
          for (int t = 0; t < TC; ++t) {
            if (kk[t] == 0) score[t] = s0;
            const uint64_t key = kk[t] >= 0 ? best_key(score[t], (uint32_t)kk[t]) : 0ull;
            best = key > best ? key : best;
          }
          rd = min(nv, rd + TC * G);
        };
        for (int c0 = 0; c0 < S; c0 += kGroupChunk<G>) {
          // one 32-bit bump word at a time (group-uniform, a broadcast read):
          // its complement is the word's valid steps, in step order, so a
          // lane's slot is the count of valid steps below its bit
#pragma unroll
          for (int wd = 0; wd < kGroupChunk<G> / 32; ++wd) {
            const int s0 = c0 + 32 * wd;
            if (s0 < S) {
              uint32_t word = ~W.BM[s0 >> 5];
              if (S - s0 < 32) word &= (1u << (S - s0)) - 1u;
#pragma unroll
              for (int h = 0; h < 32 / G; ++h) {
                const int bit = h * G + g.gl;
                if ((word >> bit) & 1u)
                  W.CK[(nv + __popc(word & below_bit[h])) & (kGroupRing<G> - 1)] =
                      (int16_t)(s0 + bit);
              }
              nv += __popc(word);
            }
          }
          wave_lds_sync();
          if (wave_ballot(nv - rd >= kGroupScoreTiles * G) != 0ull)
            pass(std::integral_constant<int, kGroupScoreTiles>{});
        }
        if (active) evals += (uint64_t)m * (uint64_t)nv;
        if (wave_ballot(nv - rd > G) != 0ull) pass(std::integral_constant<int, kGroupScoreTiles>{});
        else if (wave_ballot(nv - rd > 0) != 0ull) pass(std::integral_constant<int, 1>{});
        best = group_max_u64<G>(best);
        const int kb = best ? (int)key_index(best) : -1;
        if (g.gl == (step & (G - 1))) kreg = kb;
        if ((step & (G - 1)) == G - 1 && active) kout[(step & ~(G - 1)) + g.gl] = (int16_t)kreg;
        // apply the group's chosen angle (the voxel value from the scoring
        // expression, as rotamer_apply)
        if (kb > 0) {
          const float2 cs = A.cs[kb];
          for (int t = g.gl; t < m; t += G) {
            const int i = W.M[t];
            const Cyl c = cyl_of(W.X[i], xa, u);
            const RotBasis bs = rot_basis(c, xa, u);
            const float3 y = rot_apply(bs, cs.x, cs.y);
            // the voxel-unit basis: the one this lane stored for the step's
            // passes when they were cached (the same values), else computed
            VoxBasis vb;
            if (cached) {
              constexpr int GB = kGroupBasisAtoms<G>;
              const float *B = W.B + g.gl;
              vb = VoxBasis{B[0 * GB], B[1 * GB], B[2 * GB], B[3 * GB], B[4 * GB],
                            B[5 * GB], B[6 * GB], B[7 * GB], B[8 * GB]};
            } else {
              vb = voxel_basis(bs, GV);
            }
            const uint32_t off = basis_voxel_offset(GS, vb, cs.x, cs.y);
            W.X[i] = make_float4(y.x, y.y, y.z, GV.grid[off >> 2]);
          }
        }
        wave_lds_sync();
      }
    }
    if ((step & (G - 1)) != 0 && g.gl < (step & (G - 1)) && active)
      kout[(step & ~(G - 1)) + g.gl] = (int16_t)kreg;
    float total = 0.0f;
    for (int base = 0; base < n; base += G) {
      const int i = base + g.gl;
      total = chunk_sum_group<G>(total, i < n ? W.X[i].w : 0.0f, base, n, g.gl);
    }
    if (g.gl == 0 && active) {
      if (A.all_scores) A.all_scores[(size_t)l * O + o] = total;
      atomicMax(A.keys + l, (unsigned long long)best_key(total, (uint32_t)o));
    }
    wave_lds_sync();
  }
  if (lane == 0 && A.work) atomicAdd(A.work, (unsigned long long)kept_pairs);
  if (g.gl == 0 && A.work) atomicAdd(A.work + 1, (unsigned long long)evals);
}

template <int G, int WAVES>
static hipError_t launch_group(const SweepArgs &A, int cls, int nmax, const LaunchPlan &plan,
                               int n_cu, hipStream_t st, int *waves_per_cu) {
  const size_t shmem = (size_t)WAVES * group_wave_bytes<G>(nmax, A.S);
  *waves_per_cu = 0;
  if (shmem > 65536) return hipSuccess;
  int occ = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, sweep_group_kernel<G, WAVES>,
                                                              WAVES * kWave, shmem);
  if (e != hipSuccess) return e;
  if (occ < 1) return hipSuccess;
  const int bpc = plan.blocks_per_cu > 0 && plan.blocks_per_cu < occ ? plan.blocks_per_cu : occ;
  *waves_per_cu = bpc * WAVES;
  if (!st) return hipSuccess;  // query only
  // no more waves than the batch has units (the class sizes are only known
  // on the device; every ligand gives at most ceil(orientations / groups))
  const int64_t units = (int64_t)A.lig.n_ligands * ((A.n_orient + kWave / G - 1) / (kWave / G));
  int64_t grid = (int64_t)bpc * n_cu;
  grid = std::min<int64_t>(grid, (units + WAVES - 1) / WAVES);
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL((sweep_group_kernel<G, WAVES>), dim3((unsigned)grid), dim3(WAVES * kWave),
                     shmem, st, A, nmax, cls);
  return hipGetLastError();
}

template <int G>
static hipError_t enqueue_group_t(const SweepArgs &A, int cls, int nmax, const LaunchPlan &plan,
                                  int n_cu, hipStream_t st) {
  const int w = plan.waves_per_block;
  int n1 = 0, n2 = 0, n4 = 0;
  hipError_t e = hipSuccess;
  if (w == 4) return launch_group<G, 4>(A, cls, nmax, plan, n_cu, st, &n4);
  if (w == 2) return launch_group<G, 2>(A, cls, nmax, plan, n_cu, st, &n2);
  if (w == 1) return launch_group<G, 1>(A, cls, nmax, plan, n_cu, st, &n1);
  if (w != 0) return hipErrorInvalidValue;
  // automatic: the block size with the most resident waves (up to 6 per SIMD)
  if ((e = launch_group<G, 4>(A, cls, nmax, plan, n_cu, nullptr, &n4)) != hipSuccess) return e;
  if ((e = launch_group<G, 2>(A, cls, nmax, plan, n_cu, nullptr, &n2)) != hipSuccess) return e;
  if ((e = launch_group<G, 1>(A, cls, nmax, plan, n_cu, nullptr, &n1)) != hipSuccess) return e;
  n4 = min(n4, 24), n2 = min(n2, 24), n1 = min(n1, 24);
  if (n4 >= n2 && n4 >= n1 && n4 > 0) return launch_group<G, 4>(A, cls, nmax, plan, n_cu, st, &n4);
  if (n2 >= n1 && n2 > 0) return launch_group<G, 2>(A, cls, nmax, plan, n_cu, st, &n2);
  if (n1 > 0) return launch_group<G, 1>(A, cls, nmax, plan, n_cu, st, &n1);
  return hipErrorInvalidValue;  // not even one wave fits
}

hipError_t enqueue_sweep_group(const SweepArgs &A, int G, int cls, int nmax,
                               const LaunchPlan &plan, int n_cu, hipStream_t st) {
  if (G == 16) return enqueue_group_t<16>(A, cls, nmax, plan, n_cu, st);
  if (G == 32) return enqueue_group_t<32>(A, cls, nmax, plan, n_cu, st);
  return hipErrorInvalidValue;
}

}  // namespace dock
