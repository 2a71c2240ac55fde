// Internal types shared by the host runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sweep_common.h"

namespace dock {

constexpr int kLptBuckets = 128;  // cost buckets per size class
// Size classes of the plain sweep: ligands of at most group16 atoms are docked
// four orientations per wave (16-lane groups), those of at most group32 two
// per wave (32-lane groups), the rest one per wave; each class is a
// contiguous range of the cost-sorted ligand order with its own kernel.  The
// 32-lane ligands may be split into classes group32_split atoms wide: a
// class's LDS per wave follows its largest ligand, so the smaller ones then
// keep more resident waves (at the price of one more kernel and its tail).
//   class 0: n <= group16; 1 .. kClasses - 2: the 32-lane ligands, class
//   1 + (n - group16 - 1) / split (all in class 1 without a split);
//   kClasses - 1: the rest (one item per wave)
constexpr int kClasses = 8;
constexpr int kGroupSplitMin = 32;  // narrowest 32-lane class: at most 6 of them
constexpr int kGroupMaxAtoms16 = 96;   // largest ligands the 16-lane class may take
constexpr int kGroupMaxAtoms32 = 192;  // and the 32-lane class
// small integer block at the head of the workspace:
//   [0] work-queue counter of the one-item-per-wave sweep, [1] rejected-
//   ligand count, [4, 8) 64-bit work counters (kept pairs, evaluations),
//   [8 + c] first and [16 + c] end slot of size class c in the order,
//   [24 + c] work-queue counter of class c's grouped sweep,
//   [64, 64+B) bucket counts, [64+B, 64+2B) bucket cursors, B = 8 x 128
constexpr int kClassBegin = 8, kClassEnd = 16, kClassQueue = 24;
static_assert(kClasses <= 8, "class slots in the small block");
static_assert(kGroupMaxAtoms32 / kGroupSplitMin <= kClasses - 2, "32-lane classes");
constexpr int kSortBuckets = kClasses * kLptBuckets;
constexpr int kSmallInts = 64 + 2 * kSortBuckets;
// pruned sweep: margin (A^2) added to r_bump^2 when dropping the pairs whose
// distance lower bound shows they cannot clash
constexpr float kPruneMargin = 1e-3f;

enum SweepMode { kSweepDirect = 0, kSweepPruned = 1 };

struct LigView {
  int32_t n_ligands;
  int64_t total_atoms, total_rot, total_move;
  const int32_t *atom_offset;
  const float *xyz;
  const int32_t *rot_offset;
  const int32_t *rot_axis;
  const int32_t *move_offset;
  const int16_t *move_atoms;
};

struct SweepArgs {
  GridView grid;
  LigView lig;
  const float *orient;  // [n_orient][12], or [n_ligands][n_orient][12] per item
  int n_orient;
  int S;
  int passes;
  float r2;             // r_bump^2
  const float2 *cs;     // [S] (cos, sin) of 2 pi k / S
  const int32_t *order; // [n_ligands] ligand processed at each slot
  const int32_t *status;
  int32_t *small;       // kSmallInts counters (queue at [0])
  int32_t *queue;
  int32_t n_items;
  int32_t claim;                   // consecutive items a wave takes per queue atomic
  // work counters, accumulated once per wave: [0] kept cross pairs (summed
  // over rotamer steps), [1] (moving atom, angle) evaluations scored
  unsigned long long *work;
  unsigned long long *keys;  // [n_ligands] best (score, orientation) key
  int16_t *kstar;            // [total_rot * passes * n_orient]
  float *all_scores;         // optional [n_ligands][n_orient]
  // profile emission (learned-proposal training data), per step in the
  // layout of kstar: features [64] and score landscape [256] as BF16, and
  // the 256-bit validity mask; all NULL unless emitting
  uint16_t *emit_x;
  uint16_t *emit_t;
  uint32_t *emit_mask;
  // transforms per ligand in orient: 0 (one shared table) or n_orient (one
  // per item); last, so the fields above keep their kernel-argument offsets
  int orient_stride;
};

struct FinalOut {
  float *best_score;
  int32_t *best_orient;
  int16_t *angle_idx;
  float *xyz_out;
  int16_t *align_idx;          // optional [n_ligands]: alignment of the best orientation
  const int16_t *item_align;   // [n_ligands][n_orient] when aligned, else NULL
};

// Rigid alignment search: every (ligand, orientation) item's starting pose is
// scored under each rotation of the set (about the pose centroid) and the
// best one is folded into a per-item rigid transform for the sweep.
struct AlignArgs {
  GridView grid;
  LigView lig;
  const float *orient;     // [n_orient][12]
  int n_orient;
  const float *rot;        // [n_align][9] row-major rotations
  int n_align;
  const int32_t *status;   // [n_ligands]; items of ligands with status != 0 are skipped
  float *item_orient;      // out [n_ligands][n_orient][12]
  int16_t *item_align;     // out [n_ligands][n_orient] chosen rotation (-1: skipped)
};

struct LaunchPlan {
  int waves_per_block;  // 1, 2 or 4; 0: the one with the most resident waves
  int blocks_per_cu;    // 0 = as many as occupancy allows
  int items_per_claim;  // 1 .. 64
  int group16_atoms;    // size class docked in 16-lane groups: n <= this (0: none)
  int group32_atoms;    // size class docked in 32-lane groups: n <= this (0: none)
  int group32_split;    // width in atoms of each 32-lane class (0: one class)
};

// max_rot: ligands with more rotamers get status DOCK_E_LIMIT (at most 255).
// With lpt, ligands are ordered by size class (class bounds c16, c32: atoms
// of the 16- and 32-lane classes, 0 for none; split: the width of each
// 32-lane class, 0 for one) and, within a class, by cost;
// the class ranges go to A.small[kClassBegin/kClassEnd + c].  Without, the
// order is the input order and every ligand is in the last class.
hipError_t enqueue_prepare(const SweepArgs &A, int max_atoms, int max_rot, bool lpt, int c16,
                           int split, int c32, int32_t *bucket_of, int32_t *counts,
                           int32_t *cursor, int32_t *n_bad, hipStream_t st);
hipError_t enqueue_fill_i32(int32_t *p, int n, int32_t v, hipStream_t st);
hipError_t enqueue_sweep(const SweepArgs &A, int maxn, const LaunchPlan &plan, int n_cu,
                         hipStream_t st);
// The plain pruned sweep: with grouped classes (plan.group16/32_atoms, LPT
// order) one grouped kernel per class, then the one-item-per-wave kernel on
// the last class.
hipError_t enqueue_sweep_pruned(const SweepArgs &A, int max_atoms, const LaunchPlan &plan,
                                int n_cu, hipStream_t st);
// Grouped sweep of size class cls (G lanes per item, 64 / G items of one
// ligand per wave); nmax: the class's most atoms.
hipError_t enqueue_sweep_group(const SweepArgs &A, int G, int cls, int nmax,
                               const LaunchPlan &plan, int n_cu, hipStream_t st);
hipError_t enqueue_finalize(const SweepArgs &A, const FinalOut &F, int maxn, SweepMode mode,
                            hipStream_t st);
hipError_t enqueue_align(const AlignArgs &A, int maxn, hipStream_t st);

}  // namespace dock
