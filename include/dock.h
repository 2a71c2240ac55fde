/* dock.h -- C-ABI of the MI355X (gfx950) greedy rotamer-sweep library.
 *
 * The library implements the pose-optimisation phase of a geometric docking
 * mini-app (paper §3.1 and Listing 1: load the pocket once, then for every
 * ligand and every restart optimise the pose; §4.1 and Listing 2: every
 * fragment in sequence is rotated about its 1-D bond axis, all candidate
 * angles are evaluated in parallel and reduced to the best).
 *
 * What one (ligand, orientation) item computes:
 *   1. X = R_o X_ref + t_o                             (rigid starting pose)
 *      optional rigid alignment (paper §3.1, first phase; §4.1: rotation and
 *      scoring fused, reduced to the best, the ligand rotated once): with a
 *      rotation set R_0 .. R_{A-1}, c = mean of X,
 *        s_a = sum over atoms of grid[...] at c + R_a (X_i - c),
 *        a* = lowest a maximising s_a,  X <- c + R_a* (X - c)
 *   2. for pass in [0, passes), for rotamer r in input order:
 *        u = (X_b - X_a)/|X_b - X_a|
 *        for k in [0, S): theta_k = 2 pi k / S; Y = X with the moving atoms
 *          rotated about u through X_a (Rodrigues); k = 0 is the identity.
 *          valid_k  <=>  |Y_i - X_j|^2 >= r_bump^2 for every moving atom i
 *                        and every atom j outside the moving set and the axis
 *          s_k = sum over all atoms of grid[clamp(floor((p - o)/h))]
 *        k* = lowest k maximising s_k over valid k (-1: none, no move)
 *        X <- Y(k*)
 *   3. final score S_o = sum over atoms of the voxel values of X
 * Per ligand the best orientation (lowest index on ties) is reported with its
 * pose, score and chosen angle indices.  Arithmetic is FP32 on the GPU.
 *
 * Conventions
 *   - Every function returns DOCK_OK (0) or a negative DOCK_E_* code; no C++
 *     exception crosses this boundary.  dock_last_error() gives a
 *     thread-local detail string for the last failing call on that thread.
 *   - The caller owns every array passed in or out.  Synchronous calls keep
 *     no caller pointer after they return; asynchronous calls keep them until
 *     the stream has passed the enqueued work.
 *   - A dock_pocket owns its device copy of the grid until dock_free_pocket.
 *     One handle may be shared across threads: calls are enqueued under the
 *     handle's lock, and synchronous calls return only when done.  Work that
 *     overlaps in time on one handle must be plain-mode dock_batch_async
 *     calls on distinct streams, each with its own workspace.  Learned-mode
 *     calls, calls that pass no workspace and calls with
 *     DOCK_FLAG_TIME_SWEEP use buffers or events the handle owns and must
 *     not overlap with another such call on the same handle.
 */
#ifndef DOCK_H
#define DOCK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DOCK_OK 0
#define DOCK_E_INVAL (-1)     /* malformed argument (NULL, bad CSR, bad index) */
#define DOCK_E_LIMIT (-2)     /* outside a documented limit                    */
#define DOCK_E_NOMEM (-3)     /* device or host allocation failed              */
#define DOCK_E_DEVICE (-4)    /* HIP runtime error                             */
#define DOCK_E_CANCELLED (-5) /* reserved                                      */
#define DOCK_E_STATE (-6)     /* e.g. learned mode without a loaded proposal   */

#define DOCK_MAX_ATOMS 256    /* atoms per ligand                 */
#define DOCK_MAX_ROT 255      /* rotamers per ligand              */
#define DOCK_MAX_ALIGN 4096   /* rotations in an alignment set    */
#define DOCK_MAX_STEPS 4096   /* angle steps S                    */
#define DOCK_MAX_PASSES 16    /* refinement passes (num_repetitions) */

#define DOCK_MODE_PLAIN 0     /* full angle sweep                          */
#define DOCK_MODE_LEARNED 1   /* learned top-k proposal with full fallback */

#define DOCK_FLAG_NO_LPT 1u   /* keep input order instead of cost-sorted items */
#define DOCK_FLAG_TIME_SWEEP 2u /* record HIP events around the sweep kernel
                                   (read with dock_last_sweep_ms or
                                   dock_sweep_ms_history)                   */
#define DOCK_FLAG_DIRECT_BUMP 4u /* test every cross pair at every angle
                                    (default: only pairs that can clash)    */
#define DOCK_FLAG_GRAPH 8u       /* dock_batch_async: capture the launch
                                    sequence in a HIP graph and replay it
                                    while arguments repeat (needs a
                                    non-default stream; plain mode only:
                                    with DOCK_MODE_LEARNED, DOCK_E_INVAL)    */

typedef struct dock_pocket dock_pocket;

/* A batch of ligands in CSR form.  All indices inside a ligand are local
 * (0 .. n_l - 1).
 *   atom_offset[n_ligands+1]   ligand l owns atoms [atom_offset[l], atom_offset[l+1])
 *   xyz[total_atoms][3]        reference coordinates (A), FP32
 *   rot_offset[n_ligands+1]    ligand l owns rotamers [rot_offset[l], rot_offset[l+1])
 *   rot_axis[total_rot][2]     (a, b) axis atoms; b is on the moving side
 *   move_offset[total_rot+1]   rotamer r moves move_atoms[move_offset[r] .. move_offset[r+1])
 *                              (global positions into move_atoms)
 *   move_atoms[total_move]     local atom indices, strictly ascending per
 *                              rotamer, never a or b
 * total_* must equal atom_offset[n_ligands], rot_offset[n_ligands] and
 * move_offset[total_rot]. */
typedef struct {
  int32_t n_ligands;
  int64_t total_atoms, total_rot, total_move;
  const int32_t *atom_offset;
  const float *xyz;
  const int32_t *rot_offset;
  const int32_t *rot_axis;
  const int32_t *move_offset;
  const int16_t *move_atoms;
} dock_ligands;

typedef struct {
  float r_bump;      /* bump radius (A), >= 0                                   */
  int32_t passes;    /* sweeps over all rotamers (paper: num_repetitions), >= 1 */
  int32_t mode;      /* DOCK_MODE_PLAIN or DOCK_MODE_LEARNED                    */
  int32_t top_k;     /* learned mode: bins nominated per step (1..63); every
                        valid step of a nominated bin is scored              */
  float margin;      /* learned mode: fall back to the full sweep when the
                        predicted best minus the (top_k+1)-th is below this   */
  uint32_t flags;    /* DOCK_FLAG_*                                             */
  int32_t max_atoms; /* async calls: upper bound on atoms per ligand (0: 256)   */
  int32_t max_rot;   /* async learned calls: upper bound on rotamers, 0 .. 255
                        (0: 255); a ligand with more gets status DOCK_E_LIMIT */
  int32_t n_align;   /* rotations in the alignment set, 0 .. DOCK_MAX_ALIGN;
                        0 = no alignment (the sweep starts from R_o X_ref + t_o) */
  const float *align_rot; /* [n_align][9] row-major rotation matrices (host
                        memory for dock_batch, device memory for
                        dock_batch_async); dock_batch rejects non-finite or
                        non-orthonormal ones (|R R^T - I| > 1e-3)            */
} dock_params;

/* Outputs.  Sizes follow from the inputs.
 *   best_score[n_ligands]       FP32 final score of the best orientation
 *   best_orient[n_ligands]      its index (-1 if the ligand was rejected)
 *   angle_idx[total_rot*passes] chosen angle per step of the best
 *                               orientation; ligand l's steps start at
 *                               rot_offset[l]*passes, step = pass*R_l + r
 *   xyz_out[total_atoms][3]     final pose of the best orientation
 *   all_scores[n_ligands][n_orient]          optional (NULL): every S_o
 *   all_angle_idx[total_rot*passes*n_orient] optional (NULL): every item's
 *                               steps; (l, o) starts at
 *                               (rot_offset[l]*n_orient + o*R_l)*passes
 *   status[n_ligands]           optional (NULL): 0 or a DOCK_E_* code per
 *                               ligand (async calls validate on the device)
 *   n_fallback[n_ligands]       optional (NULL): learned mode, steps that
 *                               fell back to the full sweep
 *   align_idx[n_ligands]        optional (NULL): rotation chosen by the
 *                               alignment of the best orientation (-1 if
 *                               n_align = 0 or the ligand was rejected)
 *   all_align_idx[n_ligands][n_orient]  optional (NULL): every item's
 *                               rotation; written only when n_align > 0     */
typedef struct {
  float *best_score;
  int32_t *best_orient;
  int16_t *angle_idx;
  float *xyz_out;
  float *all_scores;
  int16_t *all_angle_idx;
  int32_t *status;
  int32_t *n_fallback;
  int16_t *align_idx;
  int16_t *all_align_idx;
} dock_results;

/* Stage a pocket grid on the current HIP device (paper Listing 1: the pocket
 * is loaded once; §4.1: the constructor copies data to the device).
 *   grid[nz][ny][nx]   host FP32 values, x fastest; voxel (ix,iy,iz) covers
 *                      origin + [i, i+1) * spacing on each axis
 *   1 <= nx,ny,nz <= 4096, nx*ny*nz < 2^30, spacing > 0.
 * On success *out owns a device copy; the host array may be freed.
 * Errors: DOCK_E_INVAL, DOCK_E_LIMIT, DOCK_E_NOMEM, DOCK_E_DEVICE. */
int dock_init_pocket(const float *grid, int nx, int ny, int nz,
                     const float origin[3], float spacing, dock_pocket **out);

/* Release a pocket and every workspace it cached.  NULL is a no-op. */
void dock_free_pocket(dock_pocket *p);

/* Synchronous batch: host arrays in, host arrays out (paper §4.1: data moves
 * once per ligand, at the start and at the end).  Inputs are validated on
 * the host first (DOCK_E_INVAL / DOCK_E_LIMIT, nothing launched).
 *   orient[n_orient][12]  rigid transforms, row-major R (9) then t (3)
 *   angle_steps           S, 1 .. DOCK_MAX_STEPS                           */
int dock_batch(dock_pocket *p, const dock_ligands *ligs, const float *orient,
               int n_orient, int angle_steps, const dock_params *prm,
               dock_results *out);

/* Device-resident batch on a caller stream (hipStream_t passed as void*,
 * NULL = default stream).  Every pointer in ligs, orient and out is a
 * device pointer; the totals in ligs must be set.  The call only enqueues
 * work and returns; results are ready when the stream reaches that point.
 * Per-ligand input errors are found on the device: such ligands are skipped,
 * get best_orient = -1 and, if out->status is set, their DOCK_E_* code.
 * workspace: device memory of at least dock_workspace_size() bytes, or NULL
 * to let the library allocate (and cache on the handle) its own.
 * Every array must be device-accessible (device, managed, pinned host or
 * unified memory): a pageable host pointer is rejected with DOCK_E_INVAL
 * before anything is enqueued. */
int dock_batch_async(dock_pocket *p, const dock_ligands *ligs,
                     const float *orient, int n_orient, int angle_steps,
                     const dock_params *prm, dock_results *out,
                     void *workspace, size_t workspace_bytes, void *stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): dock_batch_async in plain
 * mode with no workspace argument.  The workspace is a fixed device array of
 * DOCK_STATIC_SCRATCH_BYTES inside the library, one copy per device, held
 * until the process ends; its address is resolved by dock_init_pocket.  The
 * call allocates nothing (no hipMalloc, no hipFree, no allocating library
 * routine) and otherwise behaves as dock_batch_async with workspace = NULL.
 * Every call on one device shares that device's array and overwrites what
 * the previous call left there (the counters it needs zeroed are cleared by
 * the call's own kernels), so calls that overlap in time on one device race:
 * serialise them (one stream, or wait between them).
 * Errors: as dock_batch_async; DOCK_E_LIMIT when dock_workspace_size() of
 * the batch exceeds DOCK_STATIC_SCRATCH_BYTES (e.g. 10,000 ligands of 12
 * rotamers at 256 orientations need about 59 MiB); DOCK_E_INVAL for
 * DOCK_MODE_LEARNED or DOCK_FLAG_GRAPH, which allocate. */
#define DOCK_STATIC_SCRATCH_BYTES (64u << 20)
int dock_batch_async_static(dock_pocket *p, const dock_ligands *ligs,
                            const float *orient, int n_orient, int angle_steps,
                            const dock_params *prm, dock_results *out, void *stream);

/* Bytes of device workspace dock_batch_async needs for these sizes (n_align
 * as in dock_params: alignment adds 50 bytes per item). */
size_t dock_workspace_size(int32_t n_ligands, int64_t total_rot, int n_orient,
                           int angle_steps, int passes, int n_align);

/* ------------------------------------------------------------------------
 * Hybrid host + GPU docking (paper §4.2: host threads and accelerators
 * share one ligand queue; §5.1: CPU processes beside the GPU process raise
 * the node's throughput).  One dispenser hands the GPU large contiguous
 * ranges of the batch from the front (two in flight on two streams: pack,
 * copy in, sweep, copy out) and host threads a few ligands at a time from
 * the back, until the ends meet.  Host
 * threads run an FP32 CPU form of the same greedy sweep (AVX2 + FMA,
 * vectorised over angles), so each ligand's result is the GPU's or the
 * host's, equal up to FP32 rounding.
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t cpu_threads; /* host docking threads: 0 none (GPU only), -1 one per
                          hardware thread minus one (the GPU feeder's)      */
  int32_t use_gpu;     /* 1: the GPU takes chunks; 0: host threads only      */
  int32_t gpu_chunk;   /* most ligands per GPU claim (0: n_ligands/4, at
                          least 256); a claim takes a quarter of what is
                          left, at least a quarter of this cap            */
  int32_t cpu_chunk;   /* ligands per host claim (0: 1)                       */
} dock_hybrid_opts;

typedef struct {
  int64_t gpu_ligands, cpu_ligands; /* ligands docked by each side          */
  int32_t gpu_chunks, cpu_threads;  /* GPU chunks run, host threads used     */
  double wall_ms;                   /* the whole call                        */
  double gpu_busy_ms;               /* chunk times summed (copy in, sweep,
                                       copy out; the two streams overlap)    */
  double cpu_busy_ms;               /* host threads' working time, summed   */
  double feed_ms;                   /* GPU feeder packing and scattering     */
  double wait_ms;                   /* GPU feeder waiting for chunks         */
  int8_t *done_by;                  /* optional [n_ligands] (caller-owned,
                                       host): 0 GPU, 1 host thread           */
} dock_hybrid_stats;

/* Synchronous hybrid batch: host arrays in and out as in dock_batch, the
 * same validation and outputs (all_scores and all_angle_idx together or
 * neither; n_fallback, align_idx and all_align_idx are not written).  Plain
 * mode only, no alignment set (DOCK_E_INVAL otherwise).  stats may be NULL.
 * Errors: as dock_batch; DOCK_E_INVAL with use_gpu = 0 and no host
 * threads; DOCK_E_STATE when host threads are asked for on a CPU without
 * AVX2 and FMA; DOCK_E_LIMIT above 1024 threads. */
int dock_batch_hybrid(dock_pocket *p, const dock_ligands *ligs, const float *orient,
                      int n_orient, int angle_steps, const dock_params *prm,
                      dock_results *out, const dock_hybrid_opts *opt,
                      dock_hybrid_stats *stats);

/* Duration in ms of the sweep kernel of the last call on this handle that
 * set DOCK_FLAG_TIME_SWEEP (waits for that kernel to finish).  A call
 * replayed as a HIP graph (DOCK_FLAG_GRAPH) is timed around the whole graph
 * (batch preparation, alignment, sweep and finalize).  Errors:
 * DOCK_E_INVAL (NULL), DOCK_E_STATE (no timed call yet), DOCK_E_DEVICE. */
int dock_last_sweep_ms(dock_pocket *p, float *ms);

/* Sweep durations in ms of the last n calls on this handle that set
 * DOCK_FLAG_TIME_SWEEP, oldest first, into ms[0 .. n) (timed as in
 * dock_last_sweep_ms; ms[n - 1] is that function's value).  The handle keeps
 * the events of its last 16 timed calls, so a caller can enqueue up to 16
 * timed calls back to back and read them all afterwards instead of waiting
 * after each one.  Waits for the n calls' sweeps to finish.  Errors:
 * DOCK_E_INVAL (NULL, n outside [1, 16]), DOCK_E_STATE (fewer than n timed
 * calls so far), DOCK_E_DEVICE. */
int dock_sweep_ms_history(dock_pocket *p, int n, float *ms);

/* Duration in ms of the alignment kernels of the last call on this handle
 * that set DOCK_FLAG_TIME_SWEEP and n_align > 0, not replayed as a HIP graph
 * (waits for them).  Errors:
 * DOCK_E_INVAL (NULL), DOCK_E_STATE (no such call yet), DOCK_E_DEVICE. */
int dock_last_align_ms(dock_pocket *p, float *ms);

/* Work counters of the sweep kernel in the last call with
 * DOCK_FLAG_TIME_SWEEP, for roofline accounting: kept_pairs = cross pairs
 * whose clash arc was computed (those the cylinder bound could not clear),
 * summed over rotamer steps and items; atom_angle_evals = (moving atom,
 * angle) evaluations scored, i.e. sum over rotamer steps of m_r times the
 * number of non-bumping angles (every angle when emitting profiles).  Both
 * are 0 in direct-bump and learned mode.  Waits for that call's sweep.
 * Errors: DOCK_E_INVAL (NULL), DOCK_E_STATE (no timed call yet),
 * DOCK_E_DEVICE. */
int dock_last_sweep_work(dock_pocket *p, uint64_t *kept_pairs, uint64_t *atom_angle_evals);

/* Random-gather probe (benchmark instrumentation, not part of the docking
 * path): blocks x 256 threads each read iters 4-byte values at independent
 * pseudo-random offsets of buf[2^log2_floats] (device memory of at least that
 * many floats) and write one sum each to out[blocks * 256] (device memory).
 * Runs on `stream` (hipStream_t as void*, NULL = default), waits for it and
 * stores the kernel's duration in *ms.  Gathers per second =
 * blocks * 256 * iters / (ms / 1000).  Limits: 6 <= log2_floats <= 28,
 * 1 <= blocks <= 2^20, iters a multiple of 8 in [8, 65536] (DOCK_E_LIMIT);
 * NULL or host pointers: DOCK_E_INVAL. */
int dock_probe_gather(const float *buf, int log2_floats, int blocks, int iters, float *out,
                      float *ms, void *stream);

/* VALU issue probe (benchmark instrumentation, not part of the docking path):
 * blocks x 256 threads each run 8 independent dependency chains for iters
 * iterations and write one sum each to out[blocks * 256] (device memory).
 * kind 0: one FP32 FMA per chain and iteration (a = b = 1, so each sum is
 * exactly 8 iters + 8 (tid & 7) + 28 while below 2^24); kind 1: the sweep's
 * per-evaluation instruction mix, 16 VALU instructions per chain and
 * iteration (6 FMAs, 3 clamps, 3 conversions, 2 24-bit multiply-adds, a
 * conversion and an add).  Lane operations per second = blocks * 256 * 8 *
 * iters * (1 or 16) / (ms / 1000).  Runs on `stream`, waits for it and
 * stores the kernel's duration in *ms.  Limits: kind 0 or 1 (DOCK_E_INVAL),
 * 1 <= blocks <= 2^20, 1 <= iters <= 2^20 (DOCK_E_LIMIT); NULL or host
 * pointers: DOCK_E_INVAL. */
int dock_probe_valu(int kind, int blocks, int iters, float *out, float *ms, void *stream);

/* Launch mapping of the sweep kernel for calls on this handle (the knobs the
 * autotuner turns): waves_per_block in {1, 2, 4}, each wave working on its
 * own (ligand, orientation) items, or 0 (the default) for the block size that
 * keeps the most waves resident per compute unit at this batch's sizes; blocks_per_cu >= 0 caps resident blocks
 * per compute unit (0: occupancy limit); items_per_claim in [1, 64] caps how
 * many consecutive items a wave takes from the work queue per atomic (a claim
 * is a share of the items left, so it shrinks to 1 towards the end).  A new
 * handle starts at (0, 0, 16).
 * Results are bitwise identical under every mapping.  Errors: DOCK_E_INVAL. */
int dock_set_launch(dock_pocket *p, int waves_per_block, int blocks_per_cu,
                    int items_per_claim);
int dock_get_launch(dock_pocket *p, int *waves_per_block, int *blocks_per_cu,
                    int *items_per_claim);

/* Grouped mapping of the plain sweep (paper §4.1 explores gang / worker /
 * vector mappings per function; here the mapping follows the ligand's size).
 * Ligands of at most atoms16 atoms are docked four orientations per wave, one
 * 16-lane group per (ligand, orientation) item; ligands of at most atoms32
 * atoms two per wave in 32-lane groups; larger ones one per wave.  The items
 * of one wave share the ligand's topology, so the per-step bookkeeping that
 * leaves most of a 64-lane wave idle on a small ligand (clash arcs of a few
 * kept pairs, applying the chosen angle, reductions) serves several items.
 * Each size class is a contiguous range of the cost-sorted order, docked by
 * its own persistent kernel.  0 disables a class; atoms16 <= 96,
 * atoms32 <= 192 and atoms32 > atoms16 unless 0 (DOCK_E_LIMIT /
 * DOCK_E_INVAL).  Applies to plain pruned sweeps in cost order with at most
 * DOCK_GROUP_MAX_STEPS angle steps (not with DOCK_FLAG_NO_LPT or
 * DOCK_FLAG_DIRECT_BUMP, nor learned mode; above that step count scoring
 * dominates a rotamer step and one item per wave scores it faster).  Results
 * are bitwise identical under every mapping.  A new handle starts at (80, 192). */
#define DOCK_GROUP_MAX_STEPS 2048
int dock_set_group_mapping(dock_pocket *p, int atoms16, int atoms32);
int dock_get_group_mapping(dock_pocket *p, int *atoms16, int *atoms32);

/* Split of the 32-lane class: the 32-lane ligands (more than atoms16, at most
 * atoms32 atoms) are docked in classes atoms wide, (atoms16, atoms16 + atoms],
 * (atoms16 + atoms, atoms16 + 2 atoms], ..., each by a kernel of its own.  A
 * class's LDS per wave follows its largest ligand, so the smaller 32-lane
 * ligands then keep more waves resident, for the price of more kernels (and
 * the tails of their last items).  0 (a new handle's value): one 32-lane
 * class.  atoms is 0 or within [32, 192] (DOCK_E_LIMIT); NULL: DOCK_E_INVAL.
 * Results are bitwise identical either way. */
int dock_set_group_split(dock_pocket *p, int atoms);
int dock_get_group_split(dock_pocket *p, int *atoms);

/* One measured mapping of dock_autotune. */
typedef struct {
  int32_t waves_per_block, blocks_per_cu, items_per_claim;
  float sweep_ms;
  int32_t group16_atoms, group32_atoms;  /* dock_set_group_mapping's bounds */
  int32_t group32_split;                 /* dock_set_group_split's value */
} dock_tune_entry;

/* Autotuner: time the sweep for every candidate mapping (waves per block
 * 0 (automatic), 1, 2, 4 x claim caps 4, 16, 32, 64 x group bounds (0, 0), (48, 96),
 * (64, 128), (80, 128), (80, 192), and (64, 192) split every 32 atoms) on a seeded subset of
 * sample_ligands ligands of this (host) batch, keep the fastest on the handle
 * (dock_set_launch, dock_set_group_mapping, dock_set_group_split), and report each timing
 * in entries[0..*n_entries).
 * Same validation and errors as dock_batch. */
int dock_autotune(dock_pocket *p, const dock_ligands *ligs, const float *orient,
                  int n_orient, int angle_steps, const dock_params *prm,
                  int sample_ligands, uint64_t seed, dock_tune_entry *entries,
                  int max_entries, int *n_entries);

/* ------------------------------------------------------------------------
 * Learned angle proposal.  A small MLP maps 64 features of a rotamer step
 * (grid samples in the rotamer's local frame) to a 256-bin profile of the
 * angle scores; in DOCK_MODE_LEARNED the best predicted bins among the
 * angles that pass the exact bump test are scored exactly, with the full
 * sweep as fallback.  Network: 64 -> 256 -> 256 -> 256 -> 256, GELU after
 * the hidden layers, BF16 weights and activations, FP32 accumulation,
 * trained with a mean-squared error by the kernels below (all on the GPU).
 * Packed FP32 parameters (dock_mlp_param_count() floats), row-major
 * [out][in] weights: W1[256][64] b1[256] W2[256][256] b2 W3 b3 W4 b4.
 * Rows are passed as BF16 bit patterns (uint16_t), row-major; `rows` must be
 * a positive multiple of 64.  Device pointers unless stated.
 * ------------------------------------------------------------------------ */
typedef struct dock_mlp dock_mlp;

size_t dock_mlp_param_count(void);

/* Create a network on the current device from host FP32 parameters.
 * Errors: DOCK_E_INVAL, DOCK_E_NOMEM, DOCK_E_DEVICE. */
int dock_mlp_create(const float *init_params, dock_mlp **out);
void dock_mlp_free(dock_mlp *m);
int dock_mlp_get_params(dock_mlp *m, float *host_params);
int dock_mlp_set_params(dock_mlp *m, const float *host_params);

/* y[rows][256] (FP32) = network(x[rows][64]).  x and y must be
 * device-accessible (else DOCK_E_INVAL, nothing enqueued). */
int dock_mlp_forward(dock_mlp *m, const uint16_t *x_bf16, int rows, float *y, void *stream);

/* Loss = mean over rows x 256 of (y - t)^2 and its gradient w.r.t. the packed
 * parameters (kept inside the network for dock_mlp_adam; also copied to
 * grad_out if not NULL).  loss_out (host, may be NULL) waits for the stream. */
int dock_mlp_loss_grad(dock_mlp *m, const uint16_t *x_bf16, const uint16_t *t_bf16, int rows,
                       float *grad_out, float *loss_out, void *stream);

/* One Adam step (Kingma & Ba) on the FP32 master parameters with the last
 * gradient; refreshes the BF16 copy used by forward passes. */
int dock_mlp_adam(dock_mlp *m, float lr, float beta1, float beta2, float eps, void *stream);

/* Install a trained network as the pocket's learned proposal (device copy of
 * its current weights; the network may be freed afterwards).  Needed by
 * DOCK_MODE_LEARNED.  The network's 256 output bins map onto any angle_steps
 * S: bin b holds the steps of angles in [2 pi b/256, 2 pi (b+1)/256), that is
 * k in [ceil(b S/256), ceil((b+1) S/256)) (none for some bins when S < 256).
 * Learned mode requires 1 <= top_k <= 63 and top_k x ceil(S/256) + 1 <= 512;
 * otherwise DOCK_E_LIMIT. */
int dock_load_proposal(dock_pocket *p, dock_mlp *m);

/* Training data for the learned proposal: run the plain sweep (S = 256) on a
 * host batch and write, for every step of every (ligand, orientation) item
 * in the layout of all_angle_idx (item (l, o) starts at
 * (rot_offset[l]*n_orient + o*R_l)*passes), its 64 features (x_out, BF16),
 * its score landscape over the 256 angles, max(s_k - max_k' s_k', -4)
 * (t_out, BF16), and the exact validity mask of the 256 angles (mask_out,
 * 8 x uint32, bit k%32 of word k/32).  Outputs are device arrays of
 * total_rot*passes*n_orient rows. */
int dock_emit_profiles(dock_pocket *p, const dock_ligands *ligs, const float *orient,
                       int n_orient, const dock_params *prm, uint16_t *x_out,
                       uint16_t *t_out, uint32_t *mask_out);

/* Static description of a DOCK_E_* code. */
const char *dock_strerror(int code);

/* Thread-local detail of the last failing call on this thread ("" if none). */
const char *dock_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DOCK_H */
