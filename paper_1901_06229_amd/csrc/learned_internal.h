// Internal interface of the learned-proposal pipeline.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dock_internal.h"

namespace dock {

struct LearnedArgs {
  SweepArgs sw;         // grid, batch, orientations, angle table, keys, choices
  int nmax;             // LDS atoms per wave (>= largest ligand)
  float4 *pose;         // [n_items][nmax] pose between steps (x, y, z, voxel value)
  uint16_t *feat;       // [rows][64] BF16 features of each item's next step
  uint64_t *valid;      // [n_items][tiles] exact validity of the S angle steps
  const float *pred;    // [rows][256] MLP output for the current step
  int tiles;            // ceil(S / 64)
  int top_k;            // nominated bins per step (1 .. 63, top_k ceil(S / 256) < 512)
  float margin;         // fall back to the full step below this predicted margin
  int32_t *n_fallback;  // [n_ligands] steps that fell back
};

hipError_t enqueue_learned_begin(const LearnedArgs &A, int n_cu, hipStream_t st);
hipError_t enqueue_learned_step(const LearnedArgs &A, int step, int n_cu, hipStream_t st);

}  // namespace dock
