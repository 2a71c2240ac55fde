// Host form of the greedy rotamer sweep (see cpu_sweep.h).  Built with
// -mavx2 -mfma -ffp-contract=off: fused multiply-adds appear only where
// written (fmaf, _mm256_fmadd_ps), so the scalar and the 8-wide paths round
// the same way.
//
// Per (ligand, orientation) item and rotamer step (paper §3.1: fragments are
// rotated one after the other about their bond axis; §4.1: every candidate
// angle is evaluated, then reduced to the best):
//   * every atom is written in cylindrical form about the bond axis (radial
//     vector r, axial z, radius |r|);
//   * a cross pair (i moving, j static) has squared distance
//     D' - 2 (cos(theta) A + sin(theta) B), A = r_i.r_j,
//     B = u.(r_i x r_j), D' = |r_i|^2 + |r_j|^2 + (z_i - z_j)^2, never below
//     (|r_i| - |r_j|)^2 + (z_i - z_j)^2: pairs whose bound clears r_bump^2 by
//     a margin cannot bump; each other pair bumps on one open arc of angles,
//     found in closed form and marked into a bitmask of the S steps;
//   * the non-bumping steps are scored 8 at a time: per moving atom (in atom
//     order) 6 FMAs place it at the 8 angles in voxel units, then one gather;
//   * the best step (lowest index on ties) is applied and recorded.
#include "cpu_sweep.h"

#include <immintrin.h>

#include <algorithm>
#include <cmath>
#include <cstring>

namespace dock_cpu {

namespace {

constexpr float kPruneMargin = 1e-3f;  // A^2 added to r_bump^2 for the pair bound
constexpr float kStepsPerTurn = 0.15915494309189535f;  // 1 / (2 pi)

inline void mark_range(uint64_t *bits, int lo, int hi) {  // [lo, hi), 0 <= lo <= hi <= S
  while (lo < hi) {
    const int w = lo >> 6, b = lo & 63;
    const int take = std::min(64 - b, hi - lo);
    const uint64_t m = (take == 64 ? ~0ull : ((1ull << take) - 1ull)) << b;
    bits[w] |= m;
    lo += take;
  }
}

// Voxel-unit coordinate t -> cell index on an axis of n cells: clamping t to
// [0, n - 1/2] and truncating is floor-then-clamp for every finite t.
inline int cell(float t, float hi) { return (int)std::min(std::max(t, 0.0f), hi); }

}  // namespace

bool supported() {
  __builtin_cpu_init();
  return __builtin_cpu_supports("avx2") && __builtin_cpu_supports("fma");
}

// One rotamer step of the current pose; returns the chosen step (-1: none
// valid, pose unchanged).
int Worker::step(const Grid &g, const Batch &b, const Params &p, int n, int rot) {
  const int S = p.S;
  const int ra = b.rot_axis[2 * rot], rb = b.rot_axis[2 * rot + 1];
  const int m0 = b.move_offset[rot], m1 = b.move_offset[rot + 1];
  const int m = m1 - m0;
  const int16_t *mv = b.move_atoms + m0;
  const float ax = px_[ra], ay = py_[ra], az = pz_[ra];
  float ux = px_[rb] - ax, uy = py_[rb] - ay, uz = pz_[rb] - az;
  {
    const float inv = 1.0f / std::sqrt(fmaf(ux, ux, fmaf(uy, uy, uz * uz)));
    ux *= inv;
    uy *= inv;
    uz *= inv;
  }
  for (int t = 0; t < m; ++t) moving_[mv[t]] = 1;
  // cylindrical coordinates, static list, static score (atom order)
  float cst = 0.0f;
  int q = 0;
  for (int i = 0; i < n; ++i) {
    const float vx = px_[i] - ax, vy = py_[i] - ay, vz = pz_[i] - az;
    const float z = fmaf(ux, vx, fmaf(uy, vy, uz * vz));
    const float rx = fmaf(-z, ux, vx), ry = fmaf(-z, uy, vy), rz = fmaf(-z, uz, vz);
    rx_[i] = rx;
    ry_[i] = ry;
    rz_[i] = rz;
    zz_[i] = z;
    rho_[i] = std::sqrt(fmaf(rx, rx, fmaf(ry, ry, rz * rz)));
    if (!moving_[i]) {
      cst += pv_[i];
      if (i != ra && i != rb) qlist_[q++] = i;
    }
  }
  for (int t = 0; t < m; ++t) moving_[mv[t]] = 0;

  // bump mask over the S steps
  const int words = (S + 63) >> 6;
  uint64_t *bits = bump_.data();
  std::fill(bits, bits + words, 0ull);
  bool all_bump = false;
  const float thr = p.r2 + kPruneMargin;
  const float spr = (float)S * kStepsPerTurn;
  // static atoms' axial coordinates and radii, contiguous for 8-wide loads;
  // the tail is padded with an infinite radius (its bound never passes)
  float *qz = qbuf_.data(), *qr = qbuf_.data() + cap_;
  for (int t = 0; t < q; ++t) {
    qz[t] = zz_[qlist_[t]];
    qr[t] = rho_[qlist_[t]];
  }
  const int q8 = (q + 7) & ~7;
  for (int t = q; t < q8; ++t) {
    qz[t] = 0.0f;
    qr[t] = INFINITY;
  }
  const __m256 vthr = _mm256_set1_ps(thr);
  for (int t = 0; t < m && !all_bump; ++t) {
    const int i = mv[t];
    const __m256 zi = _mm256_set1_ps(zz_[i]), ri = _mm256_set1_ps(rho_[i]);
    for (int jb = 0; jb < q8 && !all_bump; jb += 8) {
      const __m256 dz = _mm256_sub_ps(zi, _mm256_loadu_ps(qz + jb));
      const __m256 dr = _mm256_sub_ps(ri, _mm256_loadu_ps(qr + jb));
      const __m256 lb = _mm256_fmadd_ps(dr, dr, _mm256_mul_ps(dz, dz));
      unsigned keep = (unsigned)_mm256_movemask_ps(_mm256_cmp_ps(lb, vthr, _CMP_LT_OQ));
      while (keep) {
        const int j = qlist_[jb + __builtin_ctz(keep)];
        keep &= keep - 1;
        // exact clash arc of the pair
        const float dzz = zz_[i] - zz_[j];
        const float A = fmaf(rx_[i], rx_[j], fmaf(ry_[i], ry_[j], rz_[i] * rz_[j]));
        const float cx = ry_[i] * rz_[j] - rz_[i] * ry_[j];
        const float cy = rz_[i] * rx_[j] - rx_[i] * rz_[j];
        const float cz = rx_[i] * ry_[j] - ry_[i] * rx_[j];
        const float B = fmaf(ux, cx, fmaf(uy, cy, uz * cz));
        const float r2i = fmaf(rx_[i], rx_[i], fmaf(ry_[i], ry_[i], rz_[i] * rz_[i]));
        const float r2j = fmaf(rx_[j], rx_[j], fmaf(ry_[j], ry_[j], rz_[j] * rz_[j]));
        const float D = fmaf(dzz, dzz, r2i + r2j) - p.r2;
        const float A2 = 2.0f * A, B2 = 2.0f * B;
        const float RR = fmaf(A2, A2, B2 * B2);
        if (D >= 0.0f && D * D >= RR) continue;  // never closer than r_bump
        if (D < 0.0f && D * D >= RR) {           // closer at every angle
          all_bump = true;
          break;
        }
        const float half = std::acos(std::min(std::max(D / std::sqrt(RR), -1.0f), 1.0f));
        const float beta = std::atan2(B2, A2);
        const int klo = (int)std::floor((beta - half) * spr) + 1;
        const int khi = (int)std::ceil((beta + half) * spr) - 1;
        const int len = khi - klo + 1;
        if (len <= 0) continue;
        if (len >= S) {
          all_bump = true;
          break;
        }
        int lo = klo % S;
        if (lo < 0) lo += S;
        const int end = lo + len;
        mark_range(bits, lo, std::min(end, S));
        if (end > S) mark_range(bits, 0, end - S);
      }
    }
  }
  if (all_bump) return -1;

  // non-bumping steps, ascending
  int nv = 0;
  for (int w = 0; w < words; ++w) {
    uint64_t free_bits = ~bits[w];
    if (w == words - 1 && (S & 63)) free_bits &= (1ull << (S & 63)) - 1ull;
    while (free_bits) {
      valid_[nv++] = (w << 6) + __builtin_ctzll(free_bits);
      free_bits &= free_bits - 1;
    }
  }
  if (nv == 0) return -1;

  // voxel-unit rotation basis of every moving atom: position on the axis
  // minus the grid corner, r and u x r, all times 1/h
  float *B = basis_.data();
  for (int t = 0; t < m; ++t) {
    const int i = mv[t];
    const float z = zz_[i];
    float *e = B + 9 * t;
    e[0] = (fmaf(z, ux, ax) - g.ox) * g.inv_h;
    e[1] = (fmaf(z, uy, ay) - g.oy) * g.inv_h;
    e[2] = (fmaf(z, uz, az) - g.oz) * g.inv_h;
    e[3] = rx_[i] * g.inv_h;
    e[4] = ry_[i] * g.inv_h;
    e[5] = rz_[i] * g.inv_h;
    e[6] = (uy * rz_[i] - uz * ry_[i]) * g.inv_h;
    e[7] = (uz * rx_[i] - ux * rz_[i]) * g.inv_h;
    e[8] = (ux * ry_[i] - uy * rx_[i]) * g.inv_h;
  }
  // step 0 (the current pose) takes the values the pose carries
  float s0 = cst;
  for (int t = 0; t < m; ++t) s0 += pv_[mv[t]];

  const __m256 hx = _mm256_set1_ps((float)g.nx - 0.5f), hy = _mm256_set1_ps((float)g.ny - 0.5f),
               hz = _mm256_set1_ps((float)g.nz - 0.5f), zero = _mm256_setzero_ps();
  const __m256i vny = _mm256_set1_epi32(g.ny), vnx = _mm256_set1_epi32(g.nx);
  float best = 0.0f;
  int kbest = -1;
  alignas(32) float cbuf[8], sbuf[8], score[8];
  for (int v0 = 0; v0 < nv; v0 += 8) {
    const int cnt = std::min(8, nv - v0);
    for (int l = 0; l < 8; ++l) {
      const int k = valid_[v0 + (l < cnt ? l : 0)];
      cbuf[l] = p.cs[2 * k];
      sbuf[l] = p.cs[2 * k + 1];
    }
    const __m256 c = _mm256_load_ps(cbuf), s = _mm256_load_ps(sbuf);
    __m256 acc = _mm256_set1_ps(cst);
    for (int t = 0; t < m; ++t) {
      const float *e = B + 9 * t;
      const __m256 tx = _mm256_fmadd_ps(s, _mm256_set1_ps(e[6]),
                                        _mm256_fmadd_ps(c, _mm256_set1_ps(e[3]), _mm256_set1_ps(e[0])));
      const __m256 ty = _mm256_fmadd_ps(s, _mm256_set1_ps(e[7]),
                                        _mm256_fmadd_ps(c, _mm256_set1_ps(e[4]), _mm256_set1_ps(e[1])));
      const __m256 tz = _mm256_fmadd_ps(s, _mm256_set1_ps(e[8]),
                                        _mm256_fmadd_ps(c, _mm256_set1_ps(e[5]), _mm256_set1_ps(e[2])));
      const __m256i ix = _mm256_cvttps_epi32(_mm256_min_ps(_mm256_max_ps(tx, zero), hx));
      const __m256i iy = _mm256_cvttps_epi32(_mm256_min_ps(_mm256_max_ps(ty, zero), hy));
      const __m256i iz = _mm256_cvttps_epi32(_mm256_min_ps(_mm256_max_ps(tz, zero), hz));
      const __m256i off = _mm256_add_epi32(
          _mm256_mullo_epi32(_mm256_add_epi32(_mm256_mullo_epi32(iz, vny), iy), vnx), ix);
      acc = _mm256_add_ps(acc, _mm256_i32gather_ps(g.v, off, 4));
    }
    _mm256_store_ps(score, acc);
    for (int l = 0; l < cnt; ++l) {
      const int k = valid_[v0 + l];
      const float sc = k == 0 ? s0 : score[l];
      if (kbest < 0 || sc > best) {
        best = sc;
        kbest = k;
      }
    }
  }
  if (kbest > 0) {
    const float c = p.cs[2 * kbest], s = p.cs[2 * kbest + 1];
    const float hxs = (float)g.nx - 0.5f, hys = (float)g.ny - 0.5f, hzs = (float)g.nz - 0.5f;
    for (int t = 0; t < m; ++t) {
      const int i = mv[t];
      const float z = zz_[i];
      const float fx = uy * rz_[i] - uz * ry_[i], fy = uz * rx_[i] - ux * rz_[i],
                  fz = ux * ry_[i] - uy * rx_[i];
      px_[i] = fmaf(s, fx, fmaf(c, rx_[i], fmaf(z, ux, ax)));
      py_[i] = fmaf(s, fy, fmaf(c, ry_[i], fmaf(z, uy, ay)));
      pz_[i] = fmaf(s, fz, fmaf(c, rz_[i], fmaf(z, uz, az)));
      // the voxel this angle was scored with (same expression as the 8-wide path)
      const float *e = B + 9 * t;
      const int ix = cell(fmaf(s, e[6], fmaf(c, e[3], e[0])), hxs);
      const int iy = cell(fmaf(s, e[7], fmaf(c, e[4], e[1])), hys);
      const int iz = cell(fmaf(s, e[8], fmaf(c, e[5], e[2])), hzs);
      pv_[i] = g.v[((size_t)iz * g.ny + iy) * g.nx + ix];
    }
  }
  return kbest;
}

void Worker::item(const Grid &g, const Batch &b, const Params &p, int l, int o, int16_t *kout) {
  const int a0 = b.atom_offset[l];
  const int n = b.atom_offset[l + 1] - a0;
  const float *T = p.orient + 12 * (size_t)o;
  const float hx = (float)g.nx - 0.5f, hy = (float)g.ny - 0.5f, hz = (float)g.nz - 0.5f;
  for (int i = 0; i < n; ++i) {
    const float *x = b.xyz + 3 * (size_t)(a0 + i);
    const float X = fmaf(T[0], x[0], fmaf(T[1], x[1], fmaf(T[2], x[2], T[9])));
    const float Y = fmaf(T[3], x[0], fmaf(T[4], x[1], fmaf(T[5], x[2], T[10])));
    const float Z = fmaf(T[6], x[0], fmaf(T[7], x[1], fmaf(T[8], x[2], T[11])));
    px_[i] = X;
    py_[i] = Y;
    pz_[i] = Z;
    const int ix = cell((X - g.ox) * g.inv_h, hx), iy = cell((Y - g.oy) * g.inv_h, hy),
              iz = cell((Z - g.oz) * g.inv_h, hz);
    pv_[i] = g.v[((size_t)iz * g.ny + iy) * g.nx + ix];
  }
  const int r0 = b.rot_offset[l], R = b.rot_offset[l + 1] - r0;
  int s = 0;
  for (int pass = 0; pass < p.passes; ++pass)
    for (int r = 0; r < R; ++r) kout[s++] = (int16_t)step(g, b, p, n, r0 + r);
}

void Worker::dock_ligand(const Grid &g, const Batch &b, const Params &p, int l, const Out &out) {
  const int a0 = b.atom_offset[l];
  const int n = b.atom_offset[l + 1] - a0;
  const int r0 = b.rot_offset[l], R = b.rot_offset[l + 1] - r0;
  const int steps = R * p.passes;
  const size_t nn = (size_t)n + 8;
  if (cap_ < nn) cap_ = nn;
  const size_t cap = cap_;
  for (auto *v : {&px_, &py_, &pz_, &pv_, &rx_, &ry_, &rz_, &zz_, &rho_})
    if (v->size() < cap) v->resize(cap);
  if (qlist_.size() < cap) qlist_.resize(cap);
  if (moving_.size() < cap) moving_.assign(cap, 0);
  if (bump_.size() < (size_t)(p.S + 63) / 64) bump_.resize((p.S + 63) / 64);
  if (valid_.size() < (size_t)p.S) valid_.resize(p.S);
  if (qbuf_.size() < 2 * cap) qbuf_.resize(2 * cap);
  if (basis_.size() < 9 * cap) basis_.resize(9 * cap);
  if (kbuf_.size() < (size_t)steps * 2 + 2) kbuf_.resize((size_t)steps * 2 + 2);
  if (best_xyz_.size() < 3 * (size_t)n) best_xyz_.resize(3 * (size_t)n);
  int16_t *kcur = kbuf_.data(), *kbest = kbuf_.data() + steps + 1;
  float best = 0.0f;
  int obest = -1;
  for (int o = 0; o < p.O; ++o) {
    int16_t *kout = out.all_angle_idx
                        ? out.all_angle_idx + ((size_t)r0 * p.O + (size_t)o * R) * p.passes
                        : kcur;
    item(g, b, p, l, o, kout);
    float total = 0.0f;
    for (int i = 0; i < n; ++i) total += pv_[i];
    if (out.all_scores) out.all_scores[(size_t)l * p.O + o] = total;
    if (obest < 0 || total > best) {
      best = total;
      obest = o;
      std::memcpy(kbest, kout, sizeof(int16_t) * steps);
      for (int i = 0; i < n; ++i) {
        best_xyz_[3 * i] = px_[i];
        best_xyz_[3 * i + 1] = py_[i];
        best_xyz_[3 * i + 2] = pz_[i];
      }
    }
  }
  out.best_score[l] = best;
  out.best_orient[l] = obest;
  if (steps) std::memcpy(out.angle_idx + (size_t)r0 * p.passes, kbest, sizeof(int16_t) * steps);
  std::memcpy(out.xyz_out + 3 * (size_t)a0, best_xyz_.data(), sizeof(float) * 3 * n);
  if (out.status) out.status[l] = 0;
}

}  // namespace dock_cpu
