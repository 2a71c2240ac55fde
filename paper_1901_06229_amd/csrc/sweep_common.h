// Device helpers shared by the sweep kernels (gfx950, wave64).
//
// Every floating-point step a pose goes through (orientation, axis,
// rotation, voxel index) lives here or in rotamer_step.h as one function.
// Within one sweep form the evaluation of an angle, the application of the
// chosen angle and the final replay of the winning orientation therefore do
// the same arithmetic: the pruned sweep scores and applies an angle through
// one voxel-space expression, the direct sweep through rodrigues and
// voxel_value.  The two forms differ from each other (and from an FP64
// evaluation) only where an atom lies within rounding of a voxel face or a
// pair within rounding of the bump radius.  The library is built with
// -ffp-contract=off; fused multiply-adds appear only where written.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dock {

constexpr int kWave = 64;

struct GridView {
  const float *grid;
  int nx, ny, nz;
  float ox, oy, oz;  // corner of voxel (0,0,0)
  float inv_h;       // 1 / spacing, rounded to FP32
};

// Cell containing p: floor((p - o)/h), clamped to the box on each axis.
__device__ __forceinline__ int voxel_index(const GridView &g, float px, float py,
                                           float pz) {
  float fx = floorf((px - g.ox) * g.inv_h);
  float fy = floorf((py - g.oy) * g.inv_h);
  float fz = floorf((pz - g.oz) * g.inv_h);
  fx = fminf(fmaxf(fx, 0.0f), (float)(g.nx - 1));
  fy = fminf(fmaxf(fy, 0.0f), (float)(g.ny - 1));
  fz = fminf(fmaxf(fz, 0.0f), (float)(g.nz - 1));
  return ((int)fz * g.ny + (int)fy) * g.nx + (int)fx;
}

__device__ __forceinline__ float voxel_value(const GridView &g, float px, float py,
                                             float pz) {
  return g.grid[voxel_index(g, px, py, pz)];
}

// Byte offset of the voxel holding a point given in voxel units ((p - o)/h).
// Clamping t to [0, n - 1/2] and truncating equals floor-then-clamp to
// [0, n - 1] for every finite t, in two instructions per axis.  Grids stay
// below 2^30 voxels, so the offset fits 32 bits and the products fit the
// 24-bit multiplier.
struct GridScaled {
  float hx, hy, hz;      // n - 1/2 per axis
  uint32_t ny, nx4;      // ny, 4 nx
};

__device__ __forceinline__ GridScaled grid_scaled(const GridView &g) {
  return GridScaled{(float)g.nx - 0.5f, (float)g.ny - 0.5f, (float)g.nz - 0.5f, (uint32_t)g.ny,
                    4u * (uint32_t)g.nx};
}

__device__ __forceinline__ uint32_t voxel_byte_offset(const GridScaled &g, float tx, float ty,
                                                      float tz) {
  const uint32_t ix = (uint32_t)__builtin_amdgcn_fmed3f(tx, 0.0f, g.hx);
  const uint32_t iy = (uint32_t)__builtin_amdgcn_fmed3f(ty, 0.0f, g.hy);
  const uint32_t iz = (uint32_t)__builtin_amdgcn_fmed3f(tz, 0.0f, g.hz);
  // Two full-rate 24-bit multiply-adds (exact: every axis has at most 4096
  // voxels).  Written out because the compiler otherwise folds the first
  // product and add into a 64-bit multiply-add, a multi-pass instruction.
  uint32_t t, off;
  asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(t) : "v"(iz), "s"(g.ny), "v"(iy));
  asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(off) : "v"(t), "s"(g.nx4), "v"(ix << 2));
  return off;
}

// Items of a persistent wave, taken from one global counter by guided
// self-scheduling: a claim is a share of the items left (as of the wave's
// previous claim) between 1 and cap, so the counter sees few atomics while
// there is much work and single items balance the tail.  The counter may end
// above n_items by at most (waves x cap); the unsigned test keeps that safe
// for any n_items < 2^31.
struct WorkQueue {
  int32_t *counter;
  int n_items, cap, share;  // share = 4 x waves in the grid
  int cur = 0, end = 0, seen = 0;
  __device__ WorkQueue(int32_t *c, int n, int cap_, int waves)
      : counter(c), n_items(n), cap(cap_), share(4 * waves) {}
  __device__ __forceinline__ bool next(int lane, int &item) {
    if (cur >= end) {
      const int want = max(1, min(cap, (n_items - seen) / share));
      int base = 0;
      if (lane == 0) base = atomicAdd(counter, want);
      base = __builtin_amdgcn_readfirstlane(__shfl(base, 0, 64));
      if ((uint32_t)base >= (uint32_t)n_items) return false;
      cur = seen = base;
      end = min(base + want, n_items);
    }
    item = cur++;
    return true;
  }
};

// Grid read through a buffer resource (32-bit offsets, reads past the end
// return 0 instead of faulting).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t grid_rsrc(const GridView &g) {
  const uint32_t bytes = 4u * (uint32_t)g.nx * (uint32_t)g.ny * (uint32_t)g.nz;
  return __builtin_amdgcn_make_buffer_rsrc((void *)g.grid, (short)0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ float grid_load(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)byte_off, 0, 0));
}

// FP32 -> BF16 bit pattern, round to nearest even.
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Value held by lane `src` (uniform) of the wave.
__device__ __forceinline__ float lane_bcast(float v, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}

// Wave ballot of a lane predicate, taken straight from the compare's lane
// mask (no select-and-compare round trip through a vector register).
__device__ __forceinline__ uint64_t wave_ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// base + the set bits of the wave-uniform mask m in the lanes below this one
// (the lane's slot in a ballot compaction): two mbcnt instructions.
__device__ __forceinline__ int lanes_before(uint64_t m, int base = 0) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                        __builtin_amdgcn_mbcnt_lo((uint32_t)m, (uint32_t)base));
}

// Rigid starting pose X = R x + t (row-major R).
__device__ __forceinline__ float3 orient_point(const float *T, float x, float y,
                                               float z) {
  float3 r;
  r.x = fmaf(T[0], x, fmaf(T[1], y, fmaf(T[2], z, T[9])));
  r.y = fmaf(T[3], x, fmaf(T[4], y, fmaf(T[5], z, T[10])));
  r.z = fmaf(T[6], x, fmaf(T[7], y, fmaf(T[8], z, T[11])));
  return r;
}

// Unit bond axis from a to b.  The hardware reciprocal square root (about
// 1 ulp) replaces an IEEE square root and divide: |u| stays within a few
// 1e-7 of 1, which moves an atom 10 A from the axis by ~1e-6 A, and every
// kernel takes the axis from here.
__device__ __forceinline__ float3 bond_axis(float4 xa, float4 xb) {
  float dx = xb.x - xa.x, dy = xb.y - xa.y, dz = xb.z - xa.z;
  float len2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
  float inv = __builtin_amdgcn_rsqf(len2);
  return make_float3(dx * inv, dy * inv, dz * inv);
}

// Rodrigues rotation of x about unit axis u through a, by the angle with
// cosine c and sine s:  Y = a + c v + s (u x v) + (1 - c)(u . v) u, v = x - a.
__device__ __forceinline__ float3 rodrigues(float4 x, float4 a, float3 u, float c,
                                            float s) {
  float vx = x.x - a.x, vy = x.y - a.y, vz = x.z - a.z;
  float cx = u.y * vz - u.z * vy;
  float cy = u.z * vx - u.x * vz;
  float cz = u.x * vy - u.y * vx;
  float udv = fmaf(u.x, vx, fmaf(u.y, vy, u.z * vz));
  float w = (1.0f - c) * udv;
  float3 y;
  y.x = fmaf(w, u.x, fmaf(s, cx, fmaf(c, vx, a.x)));
  y.y = fmaf(w, u.y, fmaf(s, cy, fmaf(c, vy, a.y)));
  y.z = fmaf(w, u.z, fmaf(s, cz, fmaf(c, vz, a.z)));
  return y;
}

// Cylindrical decomposition of x about the axis (a, u): axial coordinate
// z = (x - a).u and radial vector r = (x - a) - z u.  A rotation by theta
// moves x to  a + z u + cos(theta) r + sin(theta) (u x r)  -- the same
// Rodrigues rotation, with the parts that do not depend on theta factored
// out once per rotamer.
struct Cyl {
  float rx, ry, rz, z;
};

__device__ __forceinline__ Cyl cyl_of(float4 x, float4 a, float3 u) {
  float vx = x.x - a.x, vy = x.y - a.y, vz = x.z - a.z;
  float z = fmaf(u.x, vx, fmaf(u.y, vy, u.z * vz));
  Cyl c;
  c.rx = fmaf(-z, u.x, vx);
  c.ry = fmaf(-z, u.y, vy);
  c.rz = fmaf(-z, u.z, vz);
  c.z = z;
  return c;
}

// Angle-independent parts of the rotation of one atom: p = a + z u (on the
// axis), e = r, f = u x r.
struct RotBasis {
  float px, py, pz, ex, ey, ez, fx, fy, fz;
};

__device__ __forceinline__ RotBasis rot_basis(Cyl c, float4 a, float3 u) {
  RotBasis b;
  b.px = fmaf(c.z, u.x, a.x);
  b.py = fmaf(c.z, u.y, a.y);
  b.pz = fmaf(c.z, u.z, a.z);
  b.ex = c.rx;
  b.ey = c.ry;
  b.ez = c.rz;
  b.fx = u.y * c.rz - u.z * c.ry;
  b.fy = u.z * c.rx - u.x * c.rz;
  b.fz = u.x * c.ry - u.y * c.rx;
  return b;
}

__device__ __forceinline__ float3 rot_apply(const RotBasis &b, float c, float s) {
  return make_float3(fmaf(s, b.fx, fmaf(c, b.ex, b.px)), fmaf(s, b.fy, fmaf(c, b.ey, b.py)),
                     fmaf(s, b.fz, fmaf(c, b.ez, b.pz)));
}

// Orderable encoding of an FP32 value (monotone as an unsigned integer).
__device__ __forceinline__ uint32_t float_order(float f) {
  uint32_t b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float order_float(uint32_t o) {
  uint32_t b = (o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o;
  return __uint_as_float(b);
}

// Key for "highest score, then lowest index": (order(score), ~index).
__device__ __forceinline__ uint64_t best_key(float score, uint32_t idx) {
  return ((uint64_t)float_order(score) << 32) | (uint64_t)(0xFFFFFFFFu - idx);
}
__device__ __forceinline__ uint32_t key_index(uint64_t key) {
  return 0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFu);
}
__device__ __forceinline__ float key_score(uint64_t key) {
  return order_float((uint32_t)(key >> 32));
}

// Wave reductions with DPP lane moves (VALU, no LDS round trips).  Six
// steps combine pairs, quads, half-rows, rows, then rows 0+1 into 1 and 2+3
// into 3, then rows 0-1 into 3 (row_bcast); lane 63 ends with the result,
// which readlane hands to every lane.  The order of the combinations depends
// only on lane positions, so a floating-point sum is deterministic.  All 64
// lanes must be active.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_move(uint32_t identity, uint32_t v) {
  // lanes of rows outside ROW_MASK, or without a source lane, get identity
  return (uint32_t)__builtin_amdgcn_update_dpp((int)identity, (int)v, CTRL, ROW_MASK, 0xF, false);
}

template <class Op>
__device__ __forceinline__ uint32_t wave_reduce_bits(uint32_t v, uint32_t identity, Op op) {
  v = op(v, dpp_move<0xB1, 0xF>(identity, v));   // quad_perm [1,0,3,2]
  v = op(v, dpp_move<0x4E, 0xF>(identity, v));   // quad_perm [2,3,0,1]
  v = op(v, dpp_move<0x141, 0xF>(identity, v));  // row_half_mirror
  v = op(v, dpp_move<0x140, 0xF>(identity, v));  // row_mirror
  v = op(v, dpp_move<0x142, 0xA>(identity, v));  // row_bcast:15 into rows 1, 3
  v = op(v, dpp_move<0x143, 0xC>(identity, v));  // row_bcast:31 into rows 2, 3
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
  return wave_reduce_bits(v, 0u, [](uint32_t a, uint32_t b) { return a > b ? a : b; });
}

__device__ __forceinline__ float wave_max_f(float v) {
  return __uint_as_float(wave_reduce_bits(__float_as_uint(v), 0xFF800000u, [](uint32_t a, uint32_t b) {
    return __float_as_uint(fmaxf(__uint_as_float(a), __uint_as_float(b)));
  }));
}

__device__ __forceinline__ float wave_min_f(float v) {
  return __uint_as_float(wave_reduce_bits(__float_as_uint(v), 0x7F800000u, [](uint32_t a, uint32_t b) {
    return __float_as_uint(fminf(__uint_as_float(a), __uint_as_float(b)));
  }));
}

// Maximum 64-bit key: the high words first, then the low words of the lanes
// that hold the maximal high word.
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
  const uint32_t hi = wave_max_u32((uint32_t)(v >> 32));
  const uint32_t lo = wave_max_u32((uint32_t)(v >> 32) == hi ? (uint32_t)v : 0u);
  return ((uint64_t)hi << 32) | lo;
}

// Sum over the 64 lanes in a fixed order; every lane gets the same value.
__device__ __forceinline__ float wave_sum(float v) {
  return __uint_as_float(wave_reduce_bits(__float_as_uint(v), 0u, [](uint32_t a, uint32_t b) {
    return __float_as_uint(__uint_as_float(a) + __uint_as_float(b));
  }));
}

// Sum of the 16 lanes of each DPP row in a fixed butterfly (pairs, quads,
// half-rows, rows); every lane of the row gets the same bits (IEEE addition
// is commutative).  All lanes of the row must be active.
__device__ __forceinline__ float row_sum16(float v) {
  auto add = [](uint32_t a, uint32_t b) {
    return __float_as_uint(__uint_as_float(a) + __uint_as_float(b));
  };
  uint32_t u = __float_as_uint(v);
  u = add(u, dpp_move<0xB1, 0xF>(0u, u));   // quad_perm [1,0,3,2]
  u = add(u, dpp_move<0x4E, 0xF>(0u, u));   // quad_perm [2,3,0,1]
  u = add(u, dpp_move<0x141, 0xF>(0u, u));  // row_half_mirror
  u = add(u, dpp_move<0x140, 0xF>(0u, u));  // row_mirror
  return __uint_as_float(u);
}

// Sum over the atoms of a ligand in the order every launch mapping uses, so
// the static score and the final score are the same bits whichever mapping
// docks the item: chunks of 16 consecutive atoms are each summed by
// row_sum16 (atom 16 c + r in row lane r, absent atoms as +0), and the chunk
// sums are added one after the other in chunk order, starting from +0.
// This is the 64-lane form: lane i holds the value of atom base + i of the
// current block of 64 atoms; returns acc plus the block's chunks below n.
__device__ __forceinline__ float chunk_sum_wave(float acc, float v, int base, int n) {
  const float rs = row_sum16(v);
#pragma unroll
  for (int r = 0; r < 4; ++r)
    if (base + 16 * r < n) acc += lane_bcast(rs, 16 * r);
  return acc;
}

// Order LDS traffic between lanes of one wave (no cross-wave barrier).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

}  // namespace dock
