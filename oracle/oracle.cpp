// FP64 reference of the greedy rotamer sweep -- TEST INFRASTRUCTURE ONLY.
//
// Only the test suite, the smoke check and the benchmark's CPU-baseline leg
// load this library.  It shares no code, header or table with the GPU path;
// both read the same FP32 input arrays, which this file promotes to double.
//
// What it computes (paper §3.1 and Listing 1; the GPU formulation of the
// pose-optimisation phase in §4.1 and Listing 2):
//   for every ligand and every rigid starting pose (restart),
//     for rep in [0, passes):                        -- num_repetitions
//       for every rotamer r, in the given order      -- fragments in sequence
//         evaluate every angle of the sweep about the 1-D bond axis,
//         reject angles whose pose is not valid (intra-ligand bump),
//         score each pose with the pocket grid,
//         reduce to the best angle and apply it      -- evaluation + reduction
//   and keep the restart with the best final score.
// The paper gives no formulas; the readings used here (axis direction, angle
// grid, which pairs count as bumps, voxel rule, tie-breaks) are:
//   * axis u = (X_b - X_a)/|X_b - X_a|, right-handed angle theta about u;
//   * theta_k = 2 pi k / S, k = 0..S-1, relative to the current pose; k = 0
//     leaves the pose untouched;
//   * rotation by Rodrigues' formula, Y = X_a + c v + s (u x v) + (1-c)(u.v)u
//     with v = X - X_a;
//   * a pose is valid iff every pair (i in M_r, j in Q_r) has |Y_i - X_j|^2 >=
//     r_bump^2, where M_r is the moving set and Q_r every atom outside M_r and
//     the two axis atoms;
//   * score = sum over all atoms of grid[clamp(floor((p - o)/h))], higher is
//     better;
//   * ties: lowest angle index, lowest orientation index; no valid angle ->
//     no move, recorded as -1.
// Optional rigid alignment before the sweep (paper §3.1, first phase: the
// ligand as a rigid body is turned to the orientation that fits the pocket
// best, the score evaluated at every rotation; §4.1: rotation and scoring
// fused, a reduction to the best orientation, then one rotation of the
// ligand).  Readings:
//   * the candidate set is a caller-given list of rotation matrices R_a;
//   * each is applied about the centroid c of the starting pose,
//     Y_i = c + R_a (X_i - c), every atom moving (a rigid body keeps its
//     internal distances, so no bump test applies);
//   * score as above; the lowest index among the best scores wins.
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;

struct Pocket {
  const float *grid;
  int nx, ny, nz;
  double o[3];
  double h;
};

int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Value of the voxel containing p (cell i spans [o + i h, o + (i+1) h)).
double voxel_value(const Pocket &P, const double p[3]) {
  int n[3] = {P.nx, P.ny, P.nz};
  int idx[3];
  for (int a = 0; a < 3; ++a) {
    double f = std::floor((p[a] - P.o[a]) / P.h);
    if (f < 0) f = 0;
    if (f > n[a] - 1) f = n[a] - 1;
    idx[a] = (int)f;
  }
  return (double)P.grid[((size_t)idx[2] * P.ny + idx[1]) * P.nx + idx[0]];
}

// Range of values the voxel lookup of p can take if p moves by less than
// delta (an FP32 evaluation of the same point may land across a voxel face).
void voxel_interval(const Pocket &P, const double p[3], double delta, double *lo,
                    double *hi, bool *ambiguous) {
  int n[3] = {P.nx, P.ny, P.nz};
  int base[3], alt[3];
  bool near[3];
  for (int a = 0; a < 3; ++a) {
    double f = (p[a] - P.o[a]) / P.h;
    double fl = std::floor(f);
    base[a] = clampi((int)fl, 0, n[a] - 1);
    double d_lo = (f - fl) * P.h;        // distance to the lower face
    double d_hi = (fl + 1.0 - f) * P.h;  // distance to the upper face
    near[a] = false;
    alt[a] = base[a];
    if (d_lo < delta) {
      near[a] = true;
      alt[a] = clampi((int)fl - 1, 0, n[a] - 1);
    } else if (d_hi < delta) {
      near[a] = true;
      alt[a] = clampi((int)fl + 1, 0, n[a] - 1);
    }
  }
  double mn = 1e300, mx = -1e300;
  for (int m = 0; m < 8; ++m) {
    int idx[3];
    bool skip = false;
    for (int a = 0; a < 3; ++a) {
      bool use_alt = (m >> a) & 1;
      if (use_alt && !near[a]) skip = true;
      idx[a] = use_alt ? alt[a] : base[a];
    }
    if (skip) continue;
    double v = (double)P.grid[((size_t)idx[2] * P.ny + idx[1]) * P.nx + idx[0]];
    mn = v < mn ? v : mn;
    mx = v > mx ? v : mx;
  }
  *lo = mn;
  *hi = mx;
  *ambiguous = near[0] || near[1] || near[2];
}

// Rodrigues' rotation of x by angle (c = cos, s = sin) about the unit axis u
// through point a.
void rodrigues(const double a[3], const double u[3], double c, double s,
               const double x[3], double y[3]) {
  double v[3] = {x[0] - a[0], x[1] - a[1], x[2] - a[2]};
  double uxv[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2],
                   u[0] * v[1] - u[1] * v[0]};
  double udv = u[0] * v[0] + u[1] * v[1] + u[2] * v[2];
  for (int d = 0; d < 3; ++d)
    y[d] = a[d] + c * v[d] + s * uxv[d] + (1.0 - c) * udv * u[d];
}

struct Ligand {
  int n, R;
  const float *xyz;
  const int32_t *rot_axis;
  const int32_t *move_offset;  // local, [R+1]
  const int16_t *move_atoms;
};

// Optional per-step record (profile and ambiguity information).
struct Trace {
  const int16_t *forced_k;  // follow these choices instead of the argmax
  int forced_a;             // alignment to follow instead of the argmax (-1: none)
  double *align_s, *align_lo, *align_hi;  // [n_align]
  uint8_t *align_flags;                   // bit2 score ambiguous
  double delta;
  double *prof_s, *prof_lo, *prof_hi;  // [steps * S]
  uint8_t *prof_flags;                 // bit0 valid, bit1 validity ambiguous,
                                       // bit2 score ambiguous
  double *final_lo, *final_hi;
};

// Rigid alignment of pose X (n atoms) over the rotation set: every candidate
// scored, the best (lowest index on ties) applied about the centroid.
// Returns this reference's own argmax; the pose follows tr->forced_a if set.
int align_pose(const Pocket &P, std::vector<double> &X, int n, const float *align_rot,
               int n_align, Trace *tr) {
  double c[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < n; ++i)
    for (int d = 0; d < 3; ++d) c[d] += X[3 * i + d];
  for (int d = 0; d < 3; ++d) c[d] /= (double)n;
  auto place = [&](int a, int i, double y[3]) {
    const float *Rm = align_rot + 9 * (size_t)a;
    for (int d = 0; d < 3; ++d) {
      double acc = c[d];
      for (int e = 0; e < 3; ++e) acc += (double)Rm[3 * d + e] * (X[3 * i + e] - c[e]);
      y[d] = acc;
    }
  };
  int best_a = -1;
  double best_s = 0.0;
  for (int a = 0; a < n_align; ++a) {
    double score = 0.0, lo = 0.0, hi = 0.0;
    bool samb = false;
    for (int i = 0; i < n; ++i) {
      double y[3];
      place(a, i, y);
      score += voxel_value(P, y);
      if (tr) {
        double vl, vh;
        bool am;
        voxel_interval(P, y, tr->delta, &vl, &vh, &am);
        lo += vl;
        hi += vh;
        samb = samb || am;
      }
    }
    if (tr && tr->align_s) {
      tr->align_s[a] = score;
      tr->align_lo[a] = lo;
      tr->align_hi[a] = hi;
      tr->align_flags[a] = (uint8_t)(samb ? 4 : 0);
    }
    if (best_a < 0 || score > best_s) {
      best_a = a;
      best_s = score;
    }
  }
  const int follow = (tr && tr->forced_a >= 0) ? tr->forced_a : best_a;
  std::vector<double> Y((size_t)n * 3);
  for (int i = 0; i < n; ++i) place(follow, i, &Y[3 * i]);
  X.swap(Y);
  return best_a;
}

// One restart: orientation, optional rigid alignment, then the greedy sweep.
// Returns the final score.
double run_item(const Pocket &P, const Ligand &L, const float *orient, int S,
                double r_bump, int passes, int16_t *k_out, double *xyz_out,
                Trace *tr, const float *align_rot = nullptr, int n_align = 0,
                int16_t *a_out = nullptr) {
  const int n = L.n;
  std::vector<double> X((size_t)n * 3), Y((size_t)n * 3);
  // rigid starting pose: X = R X_ref + t
  for (int i = 0; i < n; ++i)
    for (int d = 0; d < 3; ++d) {
      double acc = (double)orient[9 + d];
      for (int e = 0; e < 3; ++e)
        acc += (double)orient[3 * d + e] * (double)L.xyz[3 * i + e];
      X[3 * i + d] = acc;
    }
  if (n_align > 0) {
    const int a = align_pose(P, X, n, align_rot, n_align, tr);
    if (a_out) *a_out = (int16_t)a;
  }
  std::vector<char> moving(n), onaxis(n);
  const double r2 = r_bump * r_bump;
  int step = 0;
  for (int pass = 0; pass < passes; ++pass) {
    for (int r = 0; r < L.R; ++r, ++step) {
      const int a = L.rot_axis[2 * r], b = L.rot_axis[2 * r + 1];
      std::fill(moving.begin(), moving.end(), 0);
      std::fill(onaxis.begin(), onaxis.end(), 0);
      onaxis[a] = onaxis[b] = 1;
      for (int t = L.move_offset[r]; t < L.move_offset[r + 1]; ++t)
        moving[L.move_atoms[t]] = 1;
      const double *Xa = &X[3 * a], *Xb = &X[3 * b];
      double u[3] = {Xb[0] - Xa[0], Xb[1] - Xa[1], Xb[2] - Xa[2]};
      double len = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
      for (int d = 0; d < 3; ++d) u[d] /= len;
      int best_k = -1;
      double best_s = 0.0;
      for (int k = 0; k < S; ++k) {
        double theta = kTwoPi * (double)k / (double)S;
        double c = std::cos(theta), s = std::sin(theta);
        // candidate pose: moving atoms rotated, everything else in place
        for (int i = 0; i < n; ++i) {
          if (moving[i] && k != 0)
            rodrigues(Xa, u, c, s, &X[3 * i], &Y[3 * i]);
          else
            for (int d = 0; d < 3; ++d) Y[3 * i + d] = X[3 * i + d];
        }
        // bump check over cross pairs M_r x Q_r
        bool valid = true, any_near = false, all_clash_near = true;
        for (int i = 0; i < n; ++i) {
          if (!moving[i]) continue;
          for (int j = 0; j < n; ++j) {
            if (moving[j] || onaxis[j]) continue;
            double dx = Y[3 * i] - X[3 * j], dy = Y[3 * i + 1] - X[3 * j + 1],
                   dz = Y[3 * i + 2] - X[3 * j + 2];
            double d2 = dx * dx + dy * dy + dz * dz;
            if (d2 < r2) {
              valid = false;
              if (!tr) break;
              if (r_bump - std::sqrt(d2) >= tr->delta) all_clash_near = false;
            } else if (tr && std::sqrt(d2) - r_bump < tr->delta) {
              any_near = true;
            }
          }
          if (!valid && !tr) break;
        }
        // score: every atom's voxel value, in atom order
        double score = 0.0, lo = 0.0, hi = 0.0;
        bool samb = false;
        for (int i = 0; i < n; ++i) {
          score += voxel_value(P, &Y[3 * i]);
          if (tr) {
            double vl, vh;
            bool am;
            voxel_interval(P, &Y[3 * i], tr->delta, &vl, &vh, &am);
            lo += vl;
            hi += vh;
            samb = samb || am;
          }
        }
        if (tr && tr->prof_s) {
          size_t at = (size_t)step * S + k;
          tr->prof_s[at] = score;
          tr->prof_lo[at] = lo;
          tr->prof_hi[at] = hi;
          bool vamb = valid ? any_near : all_clash_near;
          tr->prof_flags[at] =
              (uint8_t)((valid ? 1 : 0) | (vamb ? 2 : 0) | (samb ? 4 : 0));
        }
        // reduction: strictly greater keeps the lowest k on ties
        if (valid && (best_k < 0 || score > best_s)) {
          best_k = k;
          best_s = score;
        }
      }
      if (k_out) k_out[step] = (int16_t)best_k;
      int follow = (tr && tr->forced_k) ? tr->forced_k[step] : best_k;
      if (follow >= 0) {
        double theta = kTwoPi * (double)follow / (double)S;
        double c = std::cos(theta), s = std::sin(theta);
        for (int i = 0; i < n; ++i)
          if (moving[i] && follow != 0) {
            double y[3];
            rodrigues(Xa, u, c, s, &X[3 * i], y);
            for (int d = 0; d < 3; ++d) Y[3 * i + d] = y[d];
          }
        for (int i = 0; i < n; ++i)
          if (moving[i] && follow != 0)
            for (int d = 0; d < 3; ++d) X[3 * i + d] = Y[3 * i + d];
      }
    }
  }
  double total = 0.0, lo = 0.0, hi = 0.0;
  for (int i = 0; i < n; ++i) {
    total += voxel_value(P, &X[3 * i]);
    if (tr) {
      double vl, vh;
      bool am;
      voxel_interval(P, &X[3 * i], tr->delta, &vl, &vh, &am);
      lo += vl;
      hi += vh;
    }
  }
  if (tr && tr->final_lo) {
    *tr->final_lo = lo;
    *tr->final_hi = hi;
  }
  if (xyz_out) std::memcpy(xyz_out, X.data(), sizeof(double) * 3 * n);
  return total;
}

Pocket make_pocket(const float *grid, int nx, int ny, int nz, const float *origin,
                   float spacing) {
  Pocket P;
  P.grid = grid;
  P.nx = nx;
  P.ny = ny;
  P.nz = nz;
  for (int a = 0; a < 3; ++a) P.o[a] = (double)origin[a];
  P.h = (double)spacing;
  return P;
}

}  // namespace

extern "C" {

// Rodrigues rotation of one point (exported for the rotation pins).
void oracle_rotate(const double a[3], const double u[3], double theta,
                   const double x[3], double y[3]) {
  rodrigues(a, u, std::cos(theta), std::sin(theta), x, y);
}

double oracle_voxel_value(const float *grid, int nx, int ny, int nz,
                          const float *origin, float spacing, const double p[3]) {
  Pocket P = make_pocket(grid, nx, ny, nz, origin, spacing);
  return voxel_value(P, p);
}

// Range [lo, hi] of voxel values within delta of p, and whether p lies
// within delta of a voxel face on any axis (exported for its closed-form pins).
void oracle_voxel_interval(const float *grid, int nx, int ny, int nz,
                           const float *origin, float spacing, const double p[3],
                           double delta, double *lo, double *hi, int *ambiguous) {
  Pocket P = make_pocket(grid, nx, ny, nz, origin, spacing);
  bool am = false;
  voxel_interval(P, p, delta, lo, hi, &am);
  *ambiguous = am ? 1 : 0;
}

// One (ligand, orientation) item with the full per-step record.  forced_k
// (NULL or [passes*R]) makes the trajectory follow the given choices (used to
// replay another implementation's path); k_star always receives this
// reference's own argmax at each step of the followed trajectory.
int oracle_trace_item(const float *grid, int nx, int ny, int nz,
                      const float *origin, float spacing, int n, const float *xyz,
                      int R, const int32_t *rot_axis, const int32_t *move_offset,
                      const int16_t *move_atoms, const float *orient, int S,
                      double r_bump, int passes, const int16_t *forced_k,
                      double delta, int16_t *k_star, double *xyz_out,
                      double *final_score, double *final_lo, double *final_hi,
                      double *prof_s, double *prof_lo, double *prof_hi,
                      uint8_t *prof_flags, const float *align_rot, int n_align,
                      int forced_a, int16_t *a_star, double *align_s, double *align_lo,
                      double *align_hi, uint8_t *align_flags) {
  if (n < 1 || R < 0 || S < 1 || passes < 1 || n_align < 0) return -1;
  if (n_align > 0 && (!align_rot || forced_a >= n_align)) return -1;
  Pocket P = make_pocket(grid, nx, ny, nz, origin, spacing);
  Ligand L{n, R, xyz, rot_axis, move_offset, move_atoms};
  Trace tr{forced_k, forced_a, align_s, align_lo, align_hi, align_flags, delta,
           prof_s, prof_lo, prof_hi, prof_flags, final_lo, final_hi};
  *final_score = run_item(P, L, orient, S, r_bump, passes, k_star, xyz_out, &tr,
                          align_rot, n_align, a_star);
  return 0;
}

// Whole batch: every ligand x every orientation, best orientation per ligand.
// angle_idx: [total_rot * passes]; ligand l's entries start at
// rot_offset[l] * passes.  all_scores may be NULL.  With n_align > 0 every
// restart is aligned first; best_align[l] (may be NULL) receives the
// alignment of the best orientation, all_align[l][o] (may be NULL) every one.
int oracle_dock_batch(const float *grid, int nx, int ny, int nz,
                      const float *origin, float spacing, int n_ligands,
                      const int32_t *atom_offset, const float *xyz,
                      const int32_t *rot_offset, const int32_t *rot_axis,
                      const int32_t *move_offset, const int16_t *move_atoms,
                      const float *orient, int n_orient, int S, double r_bump,
                      int passes, double *best_score, int32_t *best_orient,
                      int16_t *angle_idx, double *xyz_out, double *all_scores,
                      int n_threads, const float *align_rot, int n_align,
                      int16_t *best_align, int16_t *all_align) {
  if (n_ligands < 0 || n_orient < 1 || S < 1 || passes < 1 || n_align < 0) return -1;
  if (n_align > 0 && !align_rot) return -1;
  Pocket P = make_pocket(grid, nx, ny, nz, origin, spacing);
  std::atomic<int> next{0};
  auto work = [&]() {
    std::vector<int32_t> moff;
    std::vector<int16_t> kbuf, kbest;
    std::vector<double> xbuf, xbest;
    for (;;) {
      int l = next.fetch_add(1);
      if (l >= n_ligands) break;
      int a0 = atom_offset[l], n = atom_offset[l + 1] - a0;
      int r0 = rot_offset[l], R = rot_offset[l + 1] - r0;
      moff.resize(R + 1);
      for (int r = 0; r <= R; ++r) moff[r] = move_offset[r0 + r] - move_offset[r0];
      Ligand L{n, R, xyz + 3 * (size_t)a0, rot_axis + 2 * (size_t)r0, moff.data(),
               move_atoms + move_offset[r0]};
      kbuf.resize((size_t)R * passes + 1);
      kbest.resize((size_t)R * passes + 1);
      xbuf.resize((size_t)n * 3);
      xbest.resize((size_t)n * 3);
      int bo = -1;
      int16_t ba = -1;
      double bs = 0.0;
      for (int o = 0; o < n_orient; ++o) {
        int16_t a = -1;
        double s = run_item(P, L, orient + 12 * (size_t)o, S, r_bump, passes,
                            kbuf.data(), xbuf.data(), nullptr, align_rot, n_align, &a);
        if (all_scores) all_scores[(size_t)l * n_orient + o] = s;
        if (all_align) all_align[(size_t)l * n_orient + o] = a;
        if (bo < 0 || s > bs) {
          bo = o;
          ba = a;
          bs = s;
          kbest.swap(kbuf);
          xbest.swap(xbuf);
        }
      }
      best_score[l] = bs;
      best_orient[l] = bo;
      if (best_align) best_align[l] = ba;
      if (angle_idx)
        std::memcpy(angle_idx + (size_t)r0 * passes, kbest.data(),
                    sizeof(int16_t) * R * passes);
      if (xyz_out)
        std::memcpy(xyz_out + 3 * (size_t)a0, xbest.data(), sizeof(double) * 3 * n);
    }
  };
  if (n_threads <= 0) n_threads = (int)std::max(1u, std::thread::hardware_concurrency());
  std::vector<std::thread> pool;
  for (int t = 1; t < n_threads; ++t) pool.emplace_back(work);
  work();
  for (auto &t : pool) t.join();
  return 0;
}

}  // extern "C"
