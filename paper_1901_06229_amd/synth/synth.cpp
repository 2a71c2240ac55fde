// Seeded synthetic inputs for the greedy rotamer sweep: pocket grids, ligand
// trees with their rotatable bonds, and rigid starting orientations.
//
// This module only *builds inputs*. It contains none of the sweep's
// arithmetic (no fragment rotation sweep, no bump test, no scoring) and is
// shared, as data, by the FP64 reference and by the GPU path.
//
// The paper does not publish its ligand library or pocket, so these recipes
// stand in for them:
//   * pocket: a G^3 FP32 grid, box centred on 0; inside the cavity the value
//     is a sum of Gaussian blobs (sigma = 2 A, amplitude U[0.5,1]), outside
//     it is -1000.  Values are sampled at voxel centres o + (i + 1/2) h.
//   * ligand: a random tree (valence <= 4) with 1.5 A bonds, bond angles
//     109.5 +- 5 deg and sibling dihedrals 120 deg apart (+- 5 deg); atoms at
//     least three bonds apart are kept >= r_bump + 0.1 A apart, so every start
//     pose is clash-free.  Rotatable bonds (rotamers) are tree edges (p, c)
//     where c has children; the moving set is the subtree beyond c.
//   * orientations: uniform random rotations (Shoemake's quaternion method),
//     translation 0 (the cavity centre).
// Randomness is counter-based: SplitMix64 keyed by (seed, stream, item), so
// ligand j is the same whatever batch it is generated in.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

namespace {

constexpr double kPi = 3.14159265358979323846;

inline uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

struct Rng {
  uint64_t s;
  Rng(uint64_t seed, uint64_t stream, uint64_t item) {
    s = mix64(mix64(mix64(seed) ^ (stream * 0xD1B54A32D192ED03ull)) ^ item);
  }
  uint64_t next() { return mix64(s += 0x632BE59BD9B4E019ull); }
  double uni() { return (double)(next() >> 11) * 0x1.0p-53; }
  double uni(double a, double b) { return a + (b - a) * uni(); }
  // inclusive integer range
  int randint(int lo, int hi) {
    return lo + (int)(next() % (uint64_t)(hi - lo + 1));
  }
  double normal() {
    double u1 = 1.0 - uni();
    double u2 = uni();
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * kPi * u2);
  }
};

struct V3 {
  double x, y, z;
};
inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
inline V3 unit(V3 a) { return (1.0 / std::sqrt(dot(a, a))) * a; }

V3 random_unit(Rng &g) {
  double z = g.uni(-1.0, 1.0);
  double t = g.uni(0.0, 2.0 * kPi);
  double r = std::sqrt(std::max(0.0, 1.0 - z * z));
  return {r * std::cos(t), r * std::sin(t), z};
}

// A unit vector perpendicular to `a` with a random phase.
V3 random_perp(Rng &g, V3 a) {
  V3 h = std::fabs(a.x) < 0.9 ? V3{1, 0, 0} : V3{0, 1, 0};
  V3 p = unit(cross(a, h));
  V3 q = cross(a, p);
  double t = g.uni(0.0, 2.0 * kPi);
  return unit(std::cos(t) * p + std::sin(t) * q);
}

// Uniform random rotation (Shoemake, "Uniform random rotations", Graphics
// Gems III, 1992): quaternion from three uniforms, then the usual matrix.
void shoemake_matrix(Rng &g, double R[9]) {
  double u1 = g.uni(), u2 = g.uni(), u3 = g.uni();
  double a = std::sqrt(1.0 - u1), b = std::sqrt(u1);
  double qx = a * std::sin(2 * kPi * u2), qy = a * std::cos(2 * kPi * u2);
  double qz = b * std::sin(2 * kPi * u3), qw = b * std::cos(2 * kPi * u3);
  R[0] = 1 - 2 * (qy * qy + qz * qz);
  R[1] = 2 * (qx * qy - qz * qw);
  R[2] = 2 * (qx * qz + qy * qw);
  R[3] = 2 * (qx * qy + qz * qw);
  R[4] = 1 - 2 * (qx * qx + qz * qz);
  R[5] = 2 * (qy * qz - qx * qw);
  R[6] = 2 * (qx * qz - qy * qw);
  R[7] = 2 * (qy * qz + qx * qw);
  R[8] = 1 - 2 * (qx * qx + qy * qy);
}

// ---------------------------------------------------------------- recipes
struct LigRecipe {
  int n_kind;   // 0 fixed, 1 uniform int, 2 lognormal(median, sigma) clipped
  double n_a, n_b;
  int n_lo, n_hi;
  int r_kind;   // 0 fixed, 1 uniform int, 2 round(40 (n-8)/142)
  int r_a, r_b;
  double chain_bias;
};

struct PocketRecipe {
  int G;
  double h;
  int n_blobs;
  int irregular;  // 0: one axis-aligned ellipsoid (10,8,6); 1: union of 4
};

bool lig_recipe(int config, LigRecipe *r) {
  switch (config) {
    case 1:
    case 4:
      *r = {0, 32, 0, 32, 32, 0, 4, 4, 0.0};
      return true;
    case 2:
      *r = {1, 20, 80, 20, 80, 1, 2, 12, 0.0};
      return true;
    case 3:
      *r = {2, 40, 0.5, 8, 150, 2, 0, 40, 0.0};
      return true;
    case 5:
      *r = {1, 100, 250, 100, 250, 1, 60, 120, 0.7};
      return true;
    default:
      return false;
  }
}

bool pocket_recipe(int config, PocketRecipe *r) {
  switch (config) {
    case 1:
    case 4:
      *r = {64, 0.5, 8, 0};
      return true;
    case 2:
    case 3:
      *r = {128, 0.375, 8, 0};
      return true;
    case 5:
      *r = {256, 0.25, 32, 1};
      return true;
    default:
      return false;
  }
}

// ---------------------------------------------------------------- ligands
struct Ligand {
  std::vector<float> xyz;           // n*3
  std::vector<int32_t> axis;        // R*2 (a, b)
  std::vector<int32_t> move_count;  // R
  std::vector<int16_t> move;        // sum of move_count
  int eligible = 0;
  int r_target = 0;
};

bool build_tree(Rng &g, int n, double chain_bias, double min_d,
                std::vector<V3> &pos, std::vector<int> &parent) {
  pos.assign(n, V3{0, 0, 0});
  parent.assign(n, -1);
  std::vector<int> deg(n, 0), nchild(n, 0), first_child(n, -1);
  std::vector<V3> wperp(n, V3{0, 0, 0});
  std::vector<double> phi0(n, 0.0);
  std::vector<int> open, bfs_dist(n), queue(n);
  std::vector<std::vector<int>> adj(n);
  phi0[0] = g.uni(0.0, 2.0 * kPi);
  for (int c = 1; c < n; ++c) {
    bool placed = false;
    for (int attempt = 0; attempt < 100 && !placed; ++attempt) {
      int p = -1;
      if (chain_bias > 0.0 && g.uni() < chain_bias && deg[c - 1] < 4) {
        p = c - 1;
      } else {
        open.clear();
        for (int x = 0; x < c; ++x)
          if (deg[x] < 4) open.push_back(x);
        if (open.empty()) return false;
        p = open[g.randint(0, (int)open.size() - 1)];
      }
      V3 d;
      if (p == 0 && nchild[0] == 0) {
        d = random_unit(g);
      } else {
        V3 bhat, w;
        int slot;
        if (parent[p] >= 0) {
          bhat = unit(pos[p] - pos[parent[p]]);
          w = wperp[p];
          slot = nchild[p];
        } else {  // root with a first child: place relative to that bond
          bhat = unit(pos[0] - pos[first_child[0]]);
          w = wperp[0];
          slot = nchild[0] - 1;
        }
        double theta = (109.5 + g.uni(-5.0, 5.0)) * kPi / 180.0;
        double phi = phi0[p] + (120.0 * slot + g.uni(-5.0, 5.0)) * kPi / 180.0;
        V3 side = std::cos(phi) * w + std::sin(phi) * cross(bhat, w);
        d = unit((-std::cos(theta)) * bhat + std::sin(theta) * side);
      }
      V3 q = pos[p] + 1.5 * d;
      // graph distances from p inside the current tree
      std::fill(bfs_dist.begin(), bfs_dist.begin() + c, -1);
      int qh = 0, qt = 0;
      queue[qt++] = p;
      bfs_dist[p] = 0;
      while (qh < qt) {
        int x = queue[qh++];
        for (int y : adj[x])
          if (bfs_dist[y] < 0) {
            bfs_dist[y] = bfs_dist[x] + 1;
            queue[qt++] = y;
          }
      }
      bool ok = true;
      for (int x = 0; x < c && ok; ++x) {
        if (bfs_dist[x] + 1 < 3) continue;  // 1-2 and 1-3 neighbours
        V3 e = q - pos[x];
        if (dot(e, e) < min_d * min_d) ok = false;
      }
      if (!ok) continue;
      pos[c] = q;
      parent[c] = p;
      adj[p].push_back(c);
      adj[c].push_back(p);
      deg[p]++;
      deg[c] = 1;
      if (nchild[p] == 0) first_child[p] = c;
      nchild[p]++;
      if (p == 0 && nchild[0] == 1) wperp[0] = random_perp(g, unit(pos[0] - q));
      wperp[c] = random_perp(g, d);
      phi0[c] = g.uni(0.0, 2.0 * kPi);
      placed = true;
    }
    if (!placed) return false;
  }
  return true;
}

int draw_n(Rng &g, const LigRecipe &r) {
  switch (r.n_kind) {
    case 0:
      return (int)r.n_a;
    case 1:
      return g.randint((int)r.n_a, (int)r.n_b);
    default: {
      double v = r.n_a * std::exp(r.n_b * g.normal());
      int n = (int)std::lround(v);
      return std::min(r.n_hi, std::max(r.n_lo, n));
    }
  }
}

int draw_r(Rng &g, const LigRecipe &r, int n) {
  switch (r.r_kind) {
    case 0:
      return r.r_a;
    case 1:
      return g.randint(r.r_a, r.r_b);
    default:
      return (int)std::lround(40.0 * (n - 8) / 142.0);
  }
}

bool make_ligand(const LigRecipe &rec, uint64_t seed, int stream, int64_t item,
                 double r_bump, Ligand *out) {
  Rng g(seed, (uint64_t)stream, (uint64_t)item);
  int n = draw_n(g, rec);
  int r_target = draw_r(g, rec, n);
  std::vector<V3> pos;
  std::vector<int> parent;
  bool ok = false;
  for (int restart = 0; restart < 1000 && !ok; ++restart)
    ok = build_tree(g, n, rec.chain_bias, r_bump + 0.1, pos, parent);
  if (!ok) return false;
  // depth and children
  std::vector<int> depth(n, 0), nchild(n, 0);
  for (int c = 1; c < n; ++c) {
    depth[c] = depth[parent[c]] + 1;
    nchild[parent[c]]++;
  }
  std::vector<int> eligible;
  for (int c = 1; c < n; ++c)
    if (nchild[c] > 0) eligible.push_back(c);
  int R = std::min(r_target, (int)eligible.size());
  R = std::max(R, 0);
  // sample R without replacement (partial Fisher-Yates)
  for (int i = 0; i < R; ++i) {
    int j = g.randint(i, (int)eligible.size() - 1);
    std::swap(eligible[i], eligible[j]);
  }
  std::vector<int> chosen(eligible.begin(), eligible.begin() + R);
  std::sort(chosen.begin(), chosen.end(), [&](int a, int b) {
    return depth[a] != depth[b] ? depth[a] < depth[b] : a < b;
  });
  // centre on the centroid
  V3 cen{0, 0, 0};
  for (int i = 0; i < n; ++i) cen = cen + pos[i];
  cen = (1.0 / n) * cen;
  out->xyz.resize((size_t)n * 3);
  for (int i = 0; i < n; ++i) {
    V3 p = pos[i] - cen;
    out->xyz[3 * i + 0] = (float)p.x;
    out->xyz[3 * i + 1] = (float)p.y;
    out->xyz[3 * i + 2] = (float)p.z;
  }
  out->axis.clear();
  out->move_count.clear();
  out->move.clear();
  std::vector<char> desc(n);
  for (int c : chosen) {
    std::fill(desc.begin(), desc.end(), 0);
    int cnt = 0;
    for (int x = c + 1; x < n; ++x) {
      // parents always precede children, so one forward pass finds the subtree
      if (parent[x] == c || (parent[x] > c && desc[parent[x]])) {
        desc[x] = 1;
        out->move.push_back((int16_t)x);
        ++cnt;
      }
    }
    out->axis.push_back(parent[c]);
    out->axis.push_back(c);
    out->move_count.push_back(cnt);
  }
  out->eligible = (int)eligible.size();
  out->r_target = r_target;
  return true;
}

struct LigandSet {
  std::vector<int32_t> atom_offset, rot_offset, rot_axis, move_offset;
  std::vector<float> xyz;
  std::vector<int16_t> move_atoms;
  std::vector<int32_t> eligible, r_target;
};

}  // namespace

extern "C" {

// Ligands [first, first+count) of (config recipe, seed, stream).  Returns an
// opaque handle (NULL on failure); read it with synth_ligands_sizes/_copy and
// release it with synth_ligands_free.
void *synth_ligands_create(int config, uint64_t seed, int stream, int64_t first,
                           int64_t count, double r_bump, int n_threads) {
  LigRecipe rec;
  if (!lig_recipe(config, &rec) || count < 0) return nullptr;
  std::vector<Ligand> ligs((size_t)count);
  std::atomic<int64_t> next{0};
  std::atomic<bool> failed{false};
  if (n_threads <= 0) n_threads = (int)std::max(1u, std::thread::hardware_concurrency());
  n_threads = (int)std::min<int64_t>(n_threads, std::max<int64_t>(1, count));
  auto work = [&]() {
    for (;;) {
      int64_t i = next.fetch_add(1);
      if (i >= count) break;
      if (!make_ligand(rec, seed, stream, first + i, r_bump, &ligs[(size_t)i]))
        failed = true;
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < n_threads; ++t) pool.emplace_back(work);
  work();
  for (auto &t : pool) t.join();
  if (failed) return nullptr;
  LigandSet *s = new (std::nothrow) LigandSet;
  if (!s) return nullptr;
  s->atom_offset.push_back(0);
  s->rot_offset.push_back(0);
  s->move_offset.push_back(0);
  for (const Ligand &L : ligs) {
    s->atom_offset.push_back(s->atom_offset.back() + (int32_t)(L.xyz.size() / 3));
    s->xyz.insert(s->xyz.end(), L.xyz.begin(), L.xyz.end());
    int R = (int)L.move_count.size();
    s->rot_offset.push_back(s->rot_offset.back() + R);
    s->rot_axis.insert(s->rot_axis.end(), L.axis.begin(), L.axis.end());
    for (int r = 0; r < R; ++r)
      s->move_offset.push_back(s->move_offset.back() + L.move_count[r]);
    s->move_atoms.insert(s->move_atoms.end(), L.move.begin(), L.move.end());
    s->eligible.push_back(L.eligible);
    s->r_target.push_back(L.r_target);
  }
  return s;
}

void synth_ligands_sizes(const void *h, int64_t *n_ligands, int64_t *total_atoms,
                         int64_t *total_rot, int64_t *total_move) {
  const LigandSet *s = (const LigandSet *)h;
  *n_ligands = (int64_t)s->atom_offset.size() - 1;
  *total_atoms = s->atom_offset.back();
  *total_rot = s->rot_offset.back();
  *total_move = s->move_offset.back();
}

void synth_ligands_copy(const void *h, int32_t *atom_offset, float *xyz,
                        int32_t *rot_offset, int32_t *rot_axis,
                        int32_t *move_offset, int16_t *move_atoms,
                        int32_t *eligible, int32_t *r_target) {
  const LigandSet *s = (const LigandSet *)h;
  auto cp = [](auto *dst, const auto &v) {
    if (dst && !v.empty()) std::memcpy(dst, v.data(), v.size() * sizeof(v[0]));
  };
  cp(atom_offset, s->atom_offset);
  cp(xyz, s->xyz);
  cp(rot_offset, s->rot_offset);
  cp(rot_axis, s->rot_axis);
  cp(move_offset, s->move_offset);
  cp(move_atoms, s->move_atoms);
  cp(eligible, s->eligible);
  cp(r_target, s->r_target);
}

void synth_ligands_free(void *h) { delete (LigandSet *)h; }

// Grid side, spacing and origin of a config's pocket (box centred on 0).
int synth_pocket_shape(int config, int *G, float *spacing, float origin[3]) {
  PocketRecipe pr;
  if (!pocket_recipe(config, &pr)) return -1;
  *G = pr.G;
  *spacing = (float)pr.h;
  for (int a = 0; a < 3; ++a) origin[a] = (float)(-0.5 * pr.G * pr.h);
  return 0;
}

// Fill grid[G^3] (x fastest) for a config's pocket recipe.
int synth_pocket_fill(int config, uint64_t seed, float *grid, int n_threads) {
  PocketRecipe pr;
  if (!pocket_recipe(config, &pr)) return -1;
  const int G = pr.G;
  const double h = pr.h, half = 0.5 * G * h;
  Rng g(seed, 0, 0);
  struct Ell {
    V3 c;
    double ax[3];
    double R[9];  // rows: body axes in world frame
  };
  std::vector<Ell> ells;
  if (!pr.irregular) {
    Ell e{{0, 0, 0}, {10, 8, 6}, {1, 0, 0, 0, 1, 0, 0, 0, 1}};
    ells.push_back(e);
  } else {
    for (int k = 0; k < 4; ++k) {
      Ell e;
      e.c = {3.0 * g.normal(), 3.0 * g.normal(), 3.0 * g.normal()};
      double cmax = std::max({std::fabs(e.c.x), std::fabs(e.c.y), std::fabs(e.c.z)});
      double lim = half - 2.0 - cmax;  // keep the ellipsoid 2 A inside the box
      for (int a = 0; a < 3; ++a) e.ax[a] = std::min(g.uni(6.0, 14.0), lim);
      shoemake_matrix(g, e.R);
      ells.push_back(e);
    }
  }
  auto inside = [&](V3 p) {
    for (const Ell &e : ells) {
      V3 d = p - e.c;
      double s = 0;
      for (int a = 0; a < 3; ++a) {
        double t = e.R[3 * a] * d.x + e.R[3 * a + 1] * d.y + e.R[3 * a + 2] * d.z;
        s += (t / e.ax[a]) * (t / e.ax[a]);
      }
      if (s <= 1.0) return true;
    }
    return false;
  };
  const double sigma = 2.0;
  std::vector<V3> mu;
  std::vector<double> amp;
  while ((int)mu.size() < pr.n_blobs) {
    V3 p{g.uni(-half, half), g.uni(-half, half), g.uni(-half, half)};
    if (!inside(p)) continue;
    mu.push_back(p);
    amp.push_back(g.uni(0.5, 1.0));
  }
  if (n_threads <= 0) n_threads = (int)std::max(1u, std::thread::hardware_concurrency());
  std::atomic<int> next{0};
  auto work = [&]() {
    for (;;) {
      int iz = next.fetch_add(1);
      if (iz >= G) break;
      for (int iy = 0; iy < G; ++iy)
        for (int ix = 0; ix < G; ++ix) {
          V3 c{-half + (ix + 0.5) * h, -half + (iy + 0.5) * h, -half + (iz + 0.5) * h};
          double v = -1000.0;
          if (inside(c)) {
            v = 0.0;
            for (size_t b = 0; b < mu.size(); ++b) {
              V3 d = c - mu[b];
              v += amp[b] * std::exp(-dot(d, d) / (2.0 * sigma * sigma));
            }
          }
          grid[((size_t)iz * G + iy) * G + ix] = (float)v;
        }
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < n_threads; ++t) pool.emplace_back(work);
  work();
  for (auto &t : pool) t.join();
  return 0;
}

// n rigid orientations [n][12] = row-major R (9) then t (3), t = 0.
int synth_orientations(uint64_t seed, int stream, int64_t first, int64_t n,
                       float *out) {
  for (int64_t o = 0; o < n; ++o) {
    Rng g(seed, (uint64_t)stream, (uint64_t)(first + o));
    double R[9];
    shoemake_matrix(g, R);
    for (int k = 0; k < 9; ++k) out[12 * o + k] = (float)R[k];
    out[12 * o + 9] = out[12 * o + 10] = out[12 * o + 11] = 0.0f;
  }
  return 0;
}

}  // extern "C"
