// Host (x86-64, AVX2 + FMA) form of the greedy rotamer sweep, used by the
// hybrid entry point: host threads take ligands from the same dispenser as
// the GPU (paper §4.2: CPU threads and the accelerator share the ligand
// queue).  FP32 throughout, like the GPU path; it is a product path of its
// own, not a reference, and shares no code with the FP64 checker.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <vector>

namespace dock_cpu {

struct Grid {
  const float *v;   // [nz][ny][nx], x fastest
  int nx, ny, nz;
  float ox, oy, oz;  // corner of voxel (0, 0, 0)
  float inv_h;       // 1 / spacing, rounded to FP32
};

// Host CSR batch (the layout of dock_ligands).
struct Batch {
  const int32_t *atom_offset;
  const float *xyz;
  const int32_t *rot_offset;
  const int32_t *rot_axis;
  const int32_t *move_offset;
  const int16_t *move_atoms;
};

// Output arrays of the whole batch (the layout of dock_results); a worker
// writes only the entries of the ligands it docks.
struct Out {
  float *best_score;
  int32_t *best_orient;
  int16_t *angle_idx;
  float *xyz_out;
  float *all_scores;       // may be NULL
  int16_t *all_angle_idx;  // may be NULL
  int32_t *status;         // may be NULL
};

struct Params {
  const float *orient;  // [O][12] row-major R then t
  int O, S, passes;
  float r2;             // r_bump^2
  const float *cs;      // [S][2] (cos, sin) of 2 pi k / S, rounded to FP32
};

// True when this CPU runs the AVX2 + FMA code.
bool supported();

// Per-thread scratch of one docking worker.
class Worker {
 public:
  // Dock ligand l over every orientation; writes its outputs.
  void dock_ligand(const Grid &g, const Batch &b, const Params &p, int l, const Out &out);

 private:
  void item(const Grid &g, const Batch &b, const Params &p, int l, int o, int16_t *kout);
  int step(const Grid &g, const Batch &b, const Params &p, int n, int rot);

  // pose of the current item: x, y, z and the voxel value carried per atom
  std::vector<float> px_, py_, pz_, pv_;
  // cylindrical coordinates about the current bond axis
  std::vector<float> rx_, ry_, rz_, zz_, rho_;
  std::vector<int> qlist_;
  std::vector<uint8_t> moving_;
  std::vector<uint64_t> bump_;  // bit k: angle step k bumps
  std::vector<int> valid_;      // non-bumping steps, ascending
  std::vector<float> qbuf_;     // static atoms' z and |r|, contiguous: [0, cap_) and [cap_, 2 cap_)
  std::vector<float> basis_;    // voxel-unit rotation basis, 9 floats per moving atom
  std::vector<float> best_xyz_;
  std::vector<int16_t> kbuf_;
  size_t cap_ = 0;              // atoms the per-atom buffers hold (n + 8)
};

}  // namespace dock_cpu
