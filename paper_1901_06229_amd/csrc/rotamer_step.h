// One rotamer step of one (ligand, orientation) item, for a 64-lane wave
// whose pose lives in LDS.  Shared by the plain sweep, the profile emitter and
// the learned-proposal kernels so all of them evaluate angles with identical
// arithmetic.
//
// Geometry of a rotation about the fixed bond axis (a, u):
//   * an atom is kept in cylindrical form, radial vector r and axial z; at
//     angle theta it sits at a + z u + cos(theta) r + sin(theta) (u x r);
//   * a cross pair (i moving, j static) has squared distance
//     D' - 2 (cos(theta) A + sin(theta) B), A = r_i.r_j, B = u.(r_i x r_j),
//     D' = |r_i|^2 + |r_j|^2 + (z_i - z_j)^2, never below
//     (|r_i| - |r_j|)^2 + (z_i - z_j)^2.  Pairs whose bound clears
//     r_bump^2 + kPruneMargin cannot bump at any angle and are dropped (the
//     bound is taken in fixed point, pack_zr below); each kept pair's clash
//     arc is marked into a bitmask of the S steps.
// Scoring takes TG angle slots per lane given by their (cos, sin); the slot-
// to-angle mapping is the caller's (compacted valid steps for the sweep,
// nominated steps for the learned proposal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dock_internal.h"
#include "sweep_common.h"

namespace dock {

constexpr int kPairCap = 128;  // LDS pair-list entries per wave

// The pair bound in fixed point.  An atom's (z, |r|) is stored as two int16
// in units of 1/256 Angstrom (truncated, saturated; z in the low half), and a
// pair's bound (dz^2 + dr^2) is one saturating packed subtract and one
// saturating integer dot product.  Truncation moves each coordinate by less
// than one unit and saturation only shortens differences, so the quantised
// distance bound stays below 256 times the float bound plus 2 sqrt(2) units.
// With the threshold widened by 3 units the test keeps every pair the float
// bound keeps (the few extra ones have empty clash arcs, so results do not
// change), in 4 bytes of LDS per atom instead of 8.
typedef short zr2_t __attribute__((ext_vector_type(2)));
constexpr float kZrUnits = 256.0f;

__device__ __forceinline__ uint32_t pack_zr(float z, float r) {
  const int zi = (int)__builtin_amdgcn_fmed3f(z * kZrUnits, -32768.0f, 32767.0f);
  const int ri = (int)fminf(r * kZrUnits, 32767.0f);  // r >= 0
  return __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pk_i16(zi, ri));
}

// quantised squared distance bound of two packed atoms (units^2)
__device__ __forceinline__ int zr_bound(uint32_t a, uint32_t b) {
  const zr2_t d = __builtin_elementwise_sub_sat(__builtin_bit_cast(zr2_t, a),
                                                __builtin_bit_cast(zr2_t, b));
  return __builtin_amdgcn_sdot2(d, d, 0, true);
}

// Pairs with zr_bound <= this may clash, for the float threshold thr
// (r_bump^2 + kPruneMargin).  Saturates to keep-everything.
__device__ __forceinline__ int zr_threshold(float thr) {
  const double b = sqrt((double)thr) * (double)kZrUnits + 3.0;
  return b * b >= 2147483647.0 ? 2147483647 : (int)(b * b) + 1;
}

// Most compacted tiles scored in one pass for a group of TG tiles: two (fewer
// live registers, 6 waves per SIMD instead of 4).  Measured on gfx950: two-
// tile passes take 4096 steps over 32-atom ligands from 4.02 M to 4.23 M
// ligands/s end to end.  Results are the same either way.
template <int TG>
constexpr int kMaxScoreTiles = TG < 2 ? TG : 2;

__host__ __device__ inline int wave_head_bytes(int nmax) {
  // X (float4), ZR (packed int16 pair), Q, M (int16), mov (uint8)
  const int b = nmax * 16 + nmax * 4 + nmax * 2 * 2 + nmax;
  return (b + 15) / 16 * 16;
}

// invalid-angle bitmask of S steps (S <= 4096)
__host__ __device__ inline int mask_bytes(int S) { return (4 * ((S + 31) / 32) + 15) / 16 * 16; }
constexpr int kBasisFloats = 9;   // voxel-space rotation basis of one atom
constexpr int kBasisBytes = kWave * kBasisFloats * 4;  // 64 atoms, component-major

// Scratch region of a wave: the kept-pair list during the bump test, then
// (when the bases are staged in LDS) the moving atoms' rotation bases and the
// compacted valid angles of a group of tg tiles while scoring.
__host__ __device__ constexpr int wave_scratch_bytes(bool lds_basis, int tg) {
  return (lds_basis ? kBasisBytes : 0) + tg * kWave * 2 > kPairCap * 4
             ? (lds_basis ? kBasisBytes : 0) + tg * kWave * 2
             : kPairCap * 4;
}

__host__ __device__ inline int wave_lds_bytes(int nmax, bool lds_basis, int tg, int S) {
  return wave_head_bytes(nmax) + wave_scratch_bytes(lds_basis, tg) + mask_bytes(S);
}

struct WaveLds {
  float4 *X;     // pose: x, y, z, voxel value
  uint32_t *ZR;  // axial coordinate and |r| about the current axis, packed
                 // for the pair bound (pack_zr); the cylindrical coordinates
                 // themselves are recomputed from X where they are needed
  int16_t *Q;    // static cross set of the rotamer
  int16_t *M;    // moving set of the rotamer
  uint8_t *mov;  // moving flags
  int *PI;       // kept pairs: i << 16 | j
  float *B;      // rotation bases of 64 moving atoms, component c of atom t at
                 // B[64 c + t] (aliases PI, used after the bump test)
  int16_t *CK;   // compacted valid angle steps (after B)
  uint32_t *BM;  // bit k set: angle step k bumps
  __device__ WaveLds(char *base, int nmax, bool lds_basis, int tg) {
    X = (float4 *)base;
    ZR = (uint32_t *)(X + nmax);
    Q = (int16_t *)(ZR + nmax);
    M = Q + nmax;
    mov = (uint8_t *)(M + nmax);
    char *scr = base + wave_head_bytes(nmax);
    PI = (int *)scr;
    B = (float *)scr;
    CK = (int16_t *)(scr + (lds_basis ? kBasisBytes : 0));
    BM = (uint32_t *)(scr + wave_scratch_bytes(lds_basis, tg));
  }
};

// |r| of an atom's cylindrical coordinates (the same expression wherever it
// is needed, so every use sees the same bits).  Hardware square root, about
// 1 ulp: the pair bound it feeds keeps a 1e-3 A^2 margin.
__device__ __forceinline__ float cyl_radius(const float4 &c) {
  return __builtin_amdgcn_sqrtf(fmaf(c.x, c.x, fmaf(c.y, c.y, c.z * c.z)));
}

struct RotState {
  int m, q;
  float cst;  // score of every atom that does not move
  float4 xa;  // axis point
  float3 u;   // unit axis
};

// Topology of one rotamer step in registers: the bond-axis atoms, the
// moving list's offset and length, and (lane t < 64) moving atom number t.
// Loaded in two parts so the sweep can fetch the next step's topology while
// it works on the current one; both are vector loads, so the waits that
// later vector loads need cover them as well.
struct RotTopo {
  int ra, rb, ms, m;
  int mv;
};

// Lanes 0-3 read ra, rb and the moving list's bounds of rotamer rot.
__device__ __forceinline__ int topo_words_load(const LigView &lig, int rot, int lane) {
  int v = 0;
  if (lane < 2)
    v = lig.rot_axis[2 * rot + lane];
  else if (lane < 4)
    v = lig.move_offset[rot + lane - 2];
  return v;
}

// Unpacks the words and loads the first 64 moving atoms.
__device__ __forceinline__ RotTopo topo_finish(const LigView &lig, int words, int lane) {
  RotTopo t;
  t.ra = __builtin_amdgcn_readlane(words, 0);
  t.rb = __builtin_amdgcn_readlane(words, 1);
  t.ms = __builtin_amdgcn_readlane(words, 2);
  t.m = __builtin_amdgcn_readlane(words, 3) - t.ms;
  t.mv = lane < t.m ? (int)lig.move_atoms[t.ms + lane] : 0;
  return t;
}

// Moving / static sets, the static score, the axis and cylindrical coords
// of the step with topology T (moving atoms past the first 64 are read from
// move_atoms).
__device__ __forceinline__ RotState rotamer_setup(const WaveLds &W, int n, const RotTopo &T,
                                                  const int16_t *move_atoms, int lane) {
  for (int i = lane; i < n; i += kWave) W.mov[i] = 0;
  wave_lds_sync();
  for (int t = lane; t < T.m; t += kWave) {
    const int i = t < kWave ? T.mv : (int)move_atoms[T.ms + t];
    W.mov[i] = 1;
    W.M[t] = (int16_t)i;
  }
  wave_lds_sync();
  RotState R;
  R.m = T.m;
  R.xa = W.X[T.ra];
  R.u = bond_axis(R.xa, W.X[T.rb]);
  // one pass over the atoms: static list, static score (the mapping-
  // independent chunked sum of chunk_sum_wave), cylindrical coordinates
  int q = 0;
  float cst = 0.0f;
  for (int base = 0; base < n; base += kWave) {
    const int i = base + lane;
    bool st = false;
    float v = 0.0f;
    if (i < n) {
      const float4 xi = W.X[i];
      const bool moving = W.mov[i] != 0;
      if (!moving) v = xi.w;
      st = !moving && i != T.ra && i != T.rb;
      const Cyl c = cyl_of(xi, R.xa, R.u);
      W.ZR[i] = pack_zr(c.z, cyl_radius(make_float4(c.rx, c.ry, c.rz, c.z)));
    }
    cst = chunk_sum_wave(cst, v, base, n);
    const uint64_t mask = wave_ballot(st);
    if (st) W.Q[lanes_before(mask, q)] = (int16_t)i;
    q += __popcll(mask);
  }
  R.q = q;
  R.cst = cst;
  wave_lds_sync();
  return R;
}

// Score of the current pose (angle step 0): static score plus the moving
// atoms' own values, added in atom order -- the order the angle scores use.
// The values are read in parallel and added by broadcast.
__device__ __forceinline__ float rotamer_s0(const WaveLds &W, const RotState &R, int lane) {
  float s = R.cst;
  for (int c0 = 0; c0 < R.m; c0 += kWave) {
    const float v = c0 + lane < R.m ? W.X[W.M[c0 + lane]].w : 0.0f;
    const int cnt = __builtin_amdgcn_readfirstlane(min(kWave, R.m - c0));  // scalar loop bound
    for (int t = 0; t < cnt; ++t) s += lane_bcast(v, t);
  }
  return s;
}

// Mark the angle steps k in [lo, hi), 0 <= lo <= hi <= S, in the bitmask.
// Word w takes the bits of [lo, hi) that fall in [32 w, 32 w + 32): both
// shift counts lie in [0, 31] for every word the loop visits.
__device__ __forceinline__ void mark_range(uint32_t *BM, int lo, int hi) {
  for (int w = lo >> 5; w <= (hi - 1) >> 5; ++w) {
    const int base = w << 5;
    atomicOr(&BM[w], (0xFFFFFFFFu << max(lo - base, 0)) & (0xFFFFFFFFu >> max(base + 32 - hi, 0)));
  }
}

// Mark the angle steps k in [lo, lo + len) (indices mod S; 0 <= lo < S,
// 0 < len <= S) in the bitmask: the part before S, then the wrapped part
// (an empty range for arcs that do not wrap).
__device__ __forceinline__ void mark_steps(uint32_t *BM, int lo, int len, int S) {
  const int end = lo + len;
  mark_range(BM, lo, min(end, S));
  mark_range(BM, 0, max(end - S, 0));
}

// Polynomial arctangent and arccosine for the clash arcs (Abramowitz and
// Stegun, Handbook of Mathematical Functions, 4.4.49 and 4.4.46: absolute
// error below 4e-8 rad in exact arithmetic, about 2.5e-7 rad evaluated in
// FP32, the size of the library routines' own rounding near pi).  An arc end
// that is off by e rad moves the pair's squared distance at that step by at
// most R e, far inside the 1e-4 A distance band the FP64 reference treats as
// ambiguous for the pair sizes of a ligand.
__device__ __forceinline__ float arc_atan2(float y, float x) {
  const float ax = fabsf(x), ay = fabsf(y);
  const float t = fminf(ax, ay) * __builtin_amdgcn_rcpf(fmaxf(ax, ay));
  const float t2 = t * t;
  float p = -0.0040540580f;
  p = fmaf(p, t2, 0.0218612288f);
  p = fmaf(p, t2, -0.0559098861f);
  p = fmaf(p, t2, 0.0964200441f);
  p = fmaf(p, t2, -0.1390853351f);
  p = fmaf(p, t2, 0.1994653599f);
  p = fmaf(p, t2, -0.3332985605f);
  p = fmaf(p, t2, 0.9999993329f);
  float a = t * p;
  a = ay > ax ? 1.57079632679f - a : a;
  a = x < 0.0f ? 3.14159265359f - a : a;
  return y < 0.0f ? -a : a;
}

__device__ __forceinline__ float arc_acos(float c) {
  const float ac = fabsf(c);
  float p = -0.0012624911f;
  p = fmaf(p, ac, 0.0066700901f);
  p = fmaf(p, ac, -0.0170881256f);
  p = fmaf(p, ac, 0.0308918810f);
  p = fmaf(p, ac, -0.0501743046f);
  p = fmaf(p, ac, 0.0889789874f);
  p = fmaf(p, ac, -0.2145988016f);
  p = fmaf(p, ac, 1.5707963050f);
  const float h = __builtin_amdgcn_sqrtf(1.0f - ac) * p;
  return c < 0.0f ? 3.14159265359f - h : h;
}

// Clash arcs of the kept pairs PI[0, cnt).  A pair bumps at angle theta iff
// cos(theta) 2A + sin(theta) 2B > D' - r^2, i.e. cos(theta - beta) > c with
// R = |(2A, 2B)|, beta = atan2(2B, 2A), c = (D' - r^2) / R: an open arc of
// half-width acos(c) around beta.  Each lane takes one pair and marks the
// angle steps inside its arc.
// The clash arc of one pair with cylindrical coordinates ci (moving) and cj
// (static) about the axis u, marked into BM (every launch mapping marks its
// kept pairs through this function).
__device__ __forceinline__ void mark_pair_arc(uint32_t *BM, const float4 &ci, const float4 &cj,
                                              const float3 &u, float r2, int S,
                                              float steps_per_rad) {
  const float dz = ci.w - cj.w;
  const float a_ = fmaf(ci.x, cj.x, fmaf(ci.y, cj.y, ci.z * cj.z));
  const float cx = ci.y * cj.z - ci.z * cj.y;
  const float cy = ci.z * cj.x - ci.x * cj.z;
  const float cz = ci.x * cj.y - ci.y * cj.x;
  const float b_ = fmaf(u.x, cx, fmaf(u.y, cy, u.z * cz));
  const float rho2i = fmaf(ci.x, ci.x, fmaf(ci.y, ci.y, ci.z * ci.z));
  const float rho2j = fmaf(cj.x, cj.x, fmaf(cj.y, cj.y, cj.z * cj.z));
  const float A2 = 2.0f * a_, B2 = 2.0f * b_;
  const float D = fmaf(dz, dz, rho2i + rho2j) - r2;
  const float RR = fmaf(A2, A2, B2 * B2);
  // |D| >= R: the sign of D decides (compared squared, no square root);
  // past these tests RR > D^2 >= 0, so the arc's R is positive
  if (D >= 0.0f && D * D >= RR) return;  // never closer than r_bump
  if (D < 0.0f && D * D >= RR) {          // closer than r_bump at every angle
    mark_steps(BM, 0, S, S);
    return;
  }
  const float half = arc_acos(__builtin_amdgcn_fmed3f(D * __builtin_amdgcn_rsqf(RR), -1.0f, 1.0f));
  const float beta = arc_atan2(B2, A2);
  const int klo = (int)floorf((beta - half) * steps_per_rad) + 1;
  const int khi = (int)ceilf((beta + half) * steps_per_rad) - 1;
  const int len = khi - klo + 1;
  if (len <= 0) return;
  if (len >= S) {
    mark_steps(BM, 0, S, S);
    return;
  }
  // klo lies in (-S, S/2 + 1]: one wrap either way replaces an integer modulo
  int lo = klo < 0 ? klo + S : klo;
  lo = lo >= S ? lo - S : lo;
  mark_steps(BM, lo, len, S);
}

__device__ __forceinline__ void mark_kept_pairs(const WaveLds &W, const RotState &R, float r2,
                                                int cnt, int S, int lane) {
  const float steps_per_rad = (float)S * 0.15915494309189535f;  // S / (2 pi)
  for (int e = lane; e < cnt; e += kWave) {
    const int ij = W.PI[e];
    const Cyl ci = cyl_of(W.X[ij >> 16], R.xa, R.u), cj = cyl_of(W.X[ij & 0xFFFF], R.xa, R.u);
    mark_pair_arc(W.BM, make_float4(ci.rx, ci.ry, ci.rz, ci.z),
                  make_float4(cj.rx, cj.ry, cj.rz, cj.z), R.u, r2, S, steps_per_rad);
  }
}

// Invalid angle steps of the rotamer, for all S steps, into W.BM.  Lanes
// sweep the flattened cross pairs (i in M, j in Q), keep those whose lower
// bound does not clear r_bump, and mark each kept pair's clash arc.  Returns
// the number of kept pairs.
__device__ __forceinline__ int rotamer_bump_mask(const WaveLds &W, const RotState &R, float r2,
                                                 int thr_q, int S, int lane) {
  for (int w = lane; w < (S + 31) / 32; w += kWave) W.BM[w] = 0u;
  int np = 0, kept = 0;
  // appends the lane's pair if act (mask: the wave's act bits); flushes the
  // list before it can overflow
  auto push = [&](uint64_t mask, bool act, int packed) {
    if (act) W.PI[lanes_before(mask, np)] = packed;
    np += __popcll(mask);
    if (np > kPairCap - kWave) {
      wave_lds_sync();
      mark_kept_pairs(W, R, r2, np, S, lane);
      kept += np;
      np = 0;
      wave_lds_sync();
    }
  };
  // lanes hold 64 static atoms; 64 moving atoms sit in registers, one per
  // lane, and are broadcast in turn
  for (int ib = 0; ib < R.m; ib += kWave) {
    // wave-uniform; kept in a scalar register so the pair loop tests it there
    const int mc = __builtin_amdgcn_readfirstlane(min(kWave, R.m - ib));
    int il = 0;
    uint32_t zl = 0u;
    if (lane < mc) {
      il = W.M[ib + lane];
      zl = W.ZR[il];
    }
    for (int jb = 0; jb < R.q; jb += kWave) {
      const bool jin = jb + lane < R.q;
      const int j = jin ? W.Q[jb + lane] : 0;
      const uint32_t zrj = W.ZR[j];
      // lanes past the static list keep nothing (bounds are never negative)
      const int tj = jin ? thr_q : -1;
      for (int t = 0; t < mc; ++t) {
        const int lb = zr_bound((uint32_t)__builtin_amdgcn_readlane((int)zl, t), zrj);
        push(wave_ballot(lb <= tj), lb <= tj,
             (__builtin_amdgcn_readlane(il, t) << 16) | j);
      }
    }
  }
  wave_lds_sync();
  mark_kept_pairs(W, R, r2, np, S, lane);
  wave_lds_sync();
  return kept + np;
}

// Wave-uniform mask of the non-bumping steps of 64-step tile `tile` (bit i:
// step 64 tile + i), zero past the S steps.  One broadcast LDS read.
__device__ __forceinline__ uint64_t tile_valid_mask(const WaveLds &W, int tile, int S) {
  const int first = tile * kWave;
  if (first >= S) return 0ull;
  const uint2 w = *(const uint2 *)(W.BM + 2 * tile);
  // readfirstlane returns int: go through uint32_t so nothing sign-extends
  const uint64_t bumps = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(w.y) << 32) |
                         (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(w.x);
  const int left = S - first;
  const uint64_t range = left >= kWave ? ~0ull : ((1ull << left) - 1ull);
  return ~bumps & range;
}

// One atom's rotation basis in voxel units relative to the grid corner:
// ((p - o)/h, e/h, f/h).  At angle (c, s) the atom's image is
// p' + c e' + s f', whose voxel is voxel_byte_offset of that point.  The
// angle scores and the application of the chosen angle both go through these
// two functions, so the voxel value a pose carries into the next step is the
// one its angle was scored with.
struct VoxBasis {
  float px, py, pz, ex, ey, ez, fx, fy, fz;
};

__device__ __forceinline__ VoxBasis voxel_basis(const RotBasis &bs, const GridView &G) {
  return VoxBasis{(bs.px - G.ox) * G.inv_h, (bs.py - G.oy) * G.inv_h, (bs.pz - G.oz) * G.inv_h,
                  bs.ex * G.inv_h,          bs.ey * G.inv_h,          bs.ez * G.inv_h,
                  bs.fx * G.inv_h,          bs.fy * G.inv_h,          bs.fz * G.inv_h};
}

__device__ __forceinline__ uint32_t basis_voxel_offset(const GridScaled &GS, const VoxBasis &b,
                                                       float c, float s) {
  return voxel_byte_offset(GS, fmaf(s, b.fx, fmaf(c, b.ex, b.px)),
                           fmaf(s, b.fy, fmaf(c, b.ey, b.py)),
                           fmaf(s, b.fz, fmaf(c, b.ez, b.pz)));
}

// Scores of the lane's TG angle slots: static score plus the voxel values
// of the rotated moving atoms, added in atom order.  Per chunk of 64 moving
// atoms each lane computes one atom's voxel-space rotation basis
// ((p - o)/h, e/h, f/h); the bases reach every lane either from LDS
// (LB: broadcast reads, no ALU work) or by readlane from the lane that holds
// them.  Gathers run one atom ahead of the adds.
template <int TG, bool LB>
__device__ __forceinline__ void rotamer_scores(const WaveLds &W, const RotState &R,
                                               const GridView &G, const GridScaled &GS,
                                               __amdgpu_buffer_rsrc_t grsrc,
                                               const float (&cc)[TG], const float (&ss)[TG],
                                               float (&score)[TG], int lane) {
#pragma unroll
  for (int t = 0; t < TG; ++t) score[t] = R.cst;
  for (int c0 = 0; c0 < R.m; c0 += kWave) {
    float b0 = 0.f, b1 = 0.f, b2 = 0.f, b3 = 0.f, b4 = 0.f, b5 = 0.f, b6 = 0.f, b7 = 0.f,
          b8 = 0.f;
    if (c0 + lane < R.m) {
      const Cyl ci = cyl_of(W.X[W.M[c0 + lane]], R.xa, R.u);
      const VoxBasis vb = voxel_basis(rot_basis(ci, R.xa, R.u), G);
      b0 = vb.px, b1 = vb.py, b2 = vb.pz;
      b3 = vb.ex, b4 = vb.ey, b5 = vb.ez;
      b6 = vb.fx, b7 = vb.fy, b8 = vb.fz;
    }
    const int cnt = min(kWave, R.m - c0);
    if constexpr (LB) {
      float *B = W.B + lane;
      B[0 * kWave] = b0, B[1 * kWave] = b1, B[2 * kWave] = b2;
      B[3 * kWave] = b3, B[4 * kWave] = b4, B[5 * kWave] = b5;
      B[6 * kWave] = b6, B[7 * kWave] = b7, B[8 * kWave] = b8;
      wave_lds_sync();
    }
    // gathers of atom tt of this chunk at the lane's TG angles
    auto gather = [&](int tt, float(&v)[TG]) {
      float px, py, pz, ex, ey, ez, fx, fy, fz;
      if constexpr (LB) {
        const float *B = W.B + tt;  // wave-uniform address: broadcast reads
        px = B[0 * kWave], py = B[1 * kWave], pz = B[2 * kWave];
        ex = B[3 * kWave], ey = B[4 * kWave], ez = B[5 * kWave];
        fx = B[6 * kWave], fy = B[7 * kWave], fz = B[8 * kWave];
      } else {
        px = lane_bcast(b0, tt), py = lane_bcast(b1, tt), pz = lane_bcast(b2, tt);
        ex = lane_bcast(b3, tt), ey = lane_bcast(b4, tt), ez = lane_bcast(b5, tt);
        fx = lane_bcast(b6, tt), fy = lane_bcast(b7, tt), fz = lane_bcast(b8, tt);
      }
      const VoxBasis vb{px, py, pz, ex, ey, ez, fx, fy, fz};
      uint32_t off[TG];
#pragma unroll
      for (int t = 0; t < TG; ++t) off[t] = basis_voxel_offset(GS, vb, cc[t], ss[t]);
#pragma unroll
      for (int t = 0; t < TG; ++t) v[t] = grid_load(grsrc, off[t]);
      __builtin_amdgcn_sched_barrier(0);  // adds stay behind these loads
    };
    auto accumulate = [&](const float(&v)[TG]) {
#pragma unroll
      for (int t = 0; t < TG; ++t) score[t] += v[t];
    };
    // two register sets alternate: atom tt + 1's gathers are issued before
    // atom tt's values are added, so no value is copied
    float va[TG], vb[TG];
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
    if constexpr (LB) wave_lds_sync();
  }
}

// Best (score, -k) key over the valid steps compacted in W.CK[0, nvalid),
// TC tiles of 64 lanes; angle step 0, if valid, is compacted first and takes
// the exact score s0 of the current pose.
template <int TC, bool LB>
__device__ __forceinline__ uint64_t score_compacted(const WaveLds &W, const RotState &R,
                                                    const GridView &G, const GridScaled &GS,
                                                    __amdgpu_buffer_rsrc_t grsrc,
                                                    const float2 *cs_table, int nvalid,
                                                    float s0, int lane, int tile0) {
  float cc[TC], ss[TC], score[TC];
  int kk[TC];
#pragma unroll
  for (int t = 0; t < TC; ++t) {
    const int j = (tile0 + t) * kWave + lane;
    kk[t] = j < nvalid ? W.CK[j] : -1;
    const float2 cs = cs_table[kk[t] > 0 ? kk[t] : 0];
    cc[t] = cs.x;
    ss[t] = cs.y;
  }
  rotamer_scores<TC, LB>(W, R, G, GS, grsrc, cc, ss, score, lane);
  uint64_t best = 0ull;
#pragma unroll
  for (int t = 0; t < TC; ++t) {
    if (kk[t] == 0) score[t] = s0;
    const uint64_t key = kk[t] >= 0 ? best_key(score[t], (uint32_t)kk[t]) : 0ull;
    best = key > best ? key : best;
  }
  return best;
}

// Scores only the valid steps of tiles t0 .. t0 + TG - 1, given their wave-
// uniform valid masks vm (bit i of vm[t]: step (t0 + t) * 64 + i): they are
// compacted into as few 64-lane tiles as possible first.  Returns the lane's
// best key (wave reduction is the caller's) and the number of valid steps in
// nvalid.
template <int TG, bool LB>
__device__ __forceinline__ uint64_t best_valid_step(const WaveLds &W, const RotState &R,
                                                    const GridView &G, const GridScaled &GS,
                                                    __amdgpu_buffer_rsrc_t grsrc,
                                                    const float2 *cs_table,
                                                    const uint64_t (&vm)[TG], int t0, float s0,
                                                    int lane, int &nvalid) {
  nvalid = 0;
#pragma unroll
  for (int t = 0; t < TG; ++t) {
    if ((vm[t] >> lane) & 1ull)
      W.CK[lanes_before(vm[t], nvalid)] = (int16_t)((t0 + t) * kWave + lane);
    nvalid += __popcll(vm[t]);
  }
  wave_lds_sync();
  uint64_t best = 0ull;
  const int tc = (nvalid + kWave - 1) / kWave;
  // one instantiation per tile count so the slot arrays stay in registers
  constexpr int MT = kMaxScoreTiles<TG>;
  for (int t0c = 0; t0c < tc; t0c += MT) {
    const int left = tc - t0c;
    uint64_t b = 0ull;
#define DOCK_SCORE_TC(c)                                                                  \
    if constexpr (MT >= c)                                                                \
      if (left == c || (c == MT && left > c))                                             \
        b = score_compacted<c, LB>(W, R, G, GS, grsrc, cs_table, nvalid, s0, lane, t0c);
    DOCK_SCORE_TC(1)
    DOCK_SCORE_TC(2)
    DOCK_SCORE_TC(3)
    DOCK_SCORE_TC(4)
    DOCK_SCORE_TC(5)
    DOCK_SCORE_TC(6)
    DOCK_SCORE_TC(7)
    DOCK_SCORE_TC(8)
#undef DOCK_SCORE_TC
    best = b > best ? b : best;
  }
  wave_lds_sync();
  return best;
}

// Rotate the moving atoms of the pose in LDS by the angle (c, s).  Each
// atom's voxel value comes from the same voxel-space expression the angle's
// score used (voxel_basis, basis_voxel_offset), not from a lookup of the
// rotated world coordinates, which can round across a voxel face differently.
__device__ __forceinline__ void rotamer_apply(const WaveLds &W, const RotState &R,
                                              const GridView &G, float c, float s, int lane) {
  const GridScaled GS = grid_scaled(G);
  for (int t = lane; t < R.m; t += kWave) {
    const int i = W.M[t];
    const RotBasis bs = rot_basis(cyl_of(W.X[i], R.xa, R.u), R.xa, R.u);
    const float3 y = rot_apply(bs, c, s);
    const uint32_t off = basis_voxel_offset(GS, voxel_basis(bs, G), c, s);
    W.X[i] = make_float4(y.x, y.y, y.z, G.grid[off >> 2]);
  }
  wave_lds_sync();
}

// The 64 input features of the learned proposal for this rotamer step: grid
// values on a 4 x 4 x 4 lattice in the rotamer's local frame -- z along the
// bond axis, x from the axis towards the moving set's centroid, y = z x x --
// spanning the swept cylinder (radius = largest |r| of the moving atoms,
// axial range [min z - 1, max z + 1]).  Values below -1 (outside the cavity)
// are clamped to -1.  Lane f computes feature f = (16 ix + 4 iy + iz).
__device__ __forceinline__ float rotamer_feature(const WaveLds &W, const RotState &R,
                                                 const GridView &G, int lane) {
  float sx = 0.f, sy = 0.f, sz = 0.f, rmax = 0.f, zmin = 3.0e38f, zmax = -3.0e38f;
  for (int t = lane; t < R.m; t += kWave) {
    const int i = W.M[t];
    const Cyl ci = cyl_of(W.X[i], R.xa, R.u);
    sx += ci.rx;
    sy += ci.ry;
    sz += ci.rz;
    rmax = fmaxf(rmax, cyl_radius(make_float4(ci.rx, ci.ry, ci.rz, ci.z)));
    zmin = fminf(zmin, ci.z);
    zmax = fmaxf(zmax, ci.z);
  }
  sx = wave_sum(sx);
  sy = wave_sum(sy);
  sz = wave_sum(sz);
  rmax = fmaxf(wave_max_f(rmax), 1e-3f);
  zmin = wave_min_f(zmin);
  zmax = wave_max_f(zmax);
  if (R.m == 0) {
    zmin = 0.0f;
    zmax = 0.0f;
  }
  const float3 u = R.u;
  float cl2 = fmaf(sx, sx, fmaf(sy, sy, sz * sz));
  if (!(cl2 > 1e-12f)) {  // no radial direction: any axis perpendicular to u
    if (fabsf(u.x) < 0.9f) {
      sx = 0.0f;
      sy = -u.z;
      sz = u.y;  // u x (1, 0, 0)
    } else {
      sx = u.z;
      sy = 0.0f;
      sz = -u.x;  // u x (0, 1, 0)
    }
    cl2 = fmaf(sx, sx, fmaf(sy, sy, sz * sz));
  }
  const float inv = 1.0f / sqrtf(cl2);
  const float ex = sx * inv, ey = sy * inv, ez = sz * inv;
  const float fx = u.y * ez - u.z * ey, fy = u.z * ex - u.x * ez, fz = u.x * ey - u.y * ex;
  const int ia = lane >> 4, ib = (lane >> 2) & 3, ic = lane & 3;
  const float lx = -rmax + 2.0f * rmax * (float)ia / 3.0f;
  const float ly = -rmax + 2.0f * rmax * (float)ib / 3.0f;
  const float z0 = zmin - 1.0f, z1 = zmax + 1.0f;
  const float lz = z0 + (z1 - z0) * (float)ic / 3.0f;
  const float px = R.xa.x + lx * ex + ly * fx + lz * u.x;
  const float py = R.xa.y + lx * ey + ly * fy + lz * u.y;
  const float pz = R.xa.z + lx * ez + ly * fz + lz * u.z;
  return fmaxf(voxel_value(G, px, py, pz), -1.0f);
}

// Final score of the pose in LDS: the chunked sum of every atom's value.
__device__ __forceinline__ float pose_total(const WaveLds &W, int n, int lane) {
  float total = 0.0f;
  for (int base = 0; base < n; base += kWave) {
    const int i = base + lane;
    total = chunk_sum_wave(total, i < n ? W.X[i].w : 0.0f, base, n);
  }
  return total;
}

// Stage the rigid starting pose (orientation T) of a ligand in LDS.
__device__ __forceinline__ void stage_pose(const WaveLds &W, const GridView &G, const float *xyz,
                                           int n, const float *T, int lane) {
  for (int i = lane; i < n; i += kWave) {
    const float *p = xyz + 3 * (size_t)i;
    const float3 x = orient_point(T, p[0], p[1], p[2]);
    W.X[i] = make_float4(x.x, x.y, x.z, voxel_value(G, x.x, x.y, x.z));
  }
  wave_lds_sync();
}

}  // namespace dock
