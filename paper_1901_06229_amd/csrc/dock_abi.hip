// Host runtime and C-ABI of the rotamer-sweep library (see include/dock.h).
//
// dock_init_pocket stages the grid once (paper Listing 1: the pocket is
// loaded before the ligand loop; §4.1: device data is owned by the object and
// copied at construction).  dock_batch moves a batch in once and the results
// out once (§4.1: data moves only at the start and the end of docking).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "dock.h"
#include <utility>

#include "abi_internal.h"
#include "dock_internal.h"
#include "learned_internal.h"
#include "mlp_internal.h"

using namespace dock;

// Timed calls whose sweep start/end events a handle keeps (dock_sweep_ms_history).
constexpr int kTimingRing = 16;

// Fixed workspace of dock_batch_async_static: one copy per device, held from
// the library's load until the process ends.  Host code never takes this
// symbol's address directly (on the host it names a stand-in, not device
// memory): dock_init_pocket resolves each device's copy once with
// hipGetSymbolAddress and the handle keeps that pointer.
static __device__ __align__(256) unsigned char scratch[DOCK_STATIC_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices] = {};

struct dock_pocket {
  int device = 0;
  float *d_grid = nullptr;
  GridView view{};
  int n_cu = 0;
  hipStream_t stream = nullptr;
  std::mutex mu;              // guards the cached buffers below
  void *ws = nullptr;         // workspace for async calls that pass none
  size_t ws_bytes = 0;
  void *io = nullptr;         // device staging of synchronous calls
  size_t io_bytes = 0;
  void *sync_ws = nullptr;    // workspace of synchronous calls
  size_t sync_ws_bytes = 0;
  // sweep start/end of the last kTimingRing timed calls; slot ring_next is
  // the next call's, ring_count of them hold a recorded call
  hipEvent_t ev_ring[kTimingRing][2] = {};
  int ring_next = 0, ring_count = 0;
  hipEvent_t ev_work = nullptr;  // the last timed call's work counters copied to h_work
  hipEvent_t ev_align[2] = {nullptr, nullptr};  // alignment start/end
  bool align_timed = false;
  unsigned long long *h_work = nullptr;  // pinned copy of the sweep's two work counters
  // grouped classes on by default: (80, 192) is within 0.2 % of the fastest
  // bounds on the 100,000-ligand uneven batch (135 ms one item per wave ->
  // 87.5 ms) and the fastest on the 10,000-ligand batch (20.6 -> 13.6 ms) and
  // on the large ligands (49.7 ms at (64, 128) -> 48.8 ms)
  LaunchPlan plan{0, 0, 16, 80, 192, 0};
  void *scratch = nullptr;    // this device's copy of the static workspace
  std::vector<float> host_grid;  // host copy of the grid, made on first use (hybrid calls)
  HybridCache hybrid;            // the hybrid entry point's streams and buffers
  // last captured launch sequence of dock_batch_async (DOCK_FLAG_GRAPH)
  std::vector<unsigned char> graph_key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  // learned proposal: BF16 weights and FP32 parameters (biases) of the MLP
  uint16_t *prop_wb = nullptr;
  float *prop_w = nullptr;
  // learned-mode buffers, grown on demand
  int64_t lw_items = 0, lw_rows = 0;
  int lw_nmax = 0, lw_tiles = 0;
  float4 *lw_pose = nullptr;
  uint16_t *lw_feat = nullptr;
  uint64_t *lw_valid = nullptr;
  float *lw_z[4] = {nullptr, nullptr, nullptr, nullptr};  // z1, z2, z3, y
  uint16_t *lw_a[3] = {nullptr, nullptr, nullptr};
  int32_t *lw_fallback = nullptr;
  int64_t lw_fallback_n = 0;
};

// The timed call just enqueued takes its ring slot.
static void ring_advance(dock_pocket *p) {
  p->ring_next = (p->ring_next + 1) % kTimingRing;
  if (p->ring_count < kTimingRing) ++p->ring_count;
}

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

}  // namespace

namespace dock {
// Shared with the other translation units of the library.
int abi_fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

// DOCK_OK if p (non-NULL) is memory the device can read and write: device,
// managed, pinned host or unified allocations.  Pageable host memory is
// rejected here, before any launch, instead of faulting a kernel.  A failed
// query leaves no sticky error behind for later launch checks.
int abi_check_device(const void *p, const char *what) {
  if (!p) return DOCK_OK;
  hipPointerAttribute_t a{};
  const hipError_t e = hipPointerGetAttributes(&a, p);
  if (e != hipSuccess) (void)hipGetLastError();
  if (e != hipSuccess || (a.type != hipMemoryTypeDevice && a.type != hipMemoryTypeManaged &&
                          a.type != hipMemoryTypeHost && a.type != hipMemoryTypeUnified))
    return abi_fail(DOCK_E_INVAL, "%s is not device-accessible memory", what);
  return DOCK_OK;
}
}  // namespace dock

namespace {

int hip_fail(hipError_t e, const char *what) {
  return fail(e == hipErrorOutOfMemory ? DOCK_E_NOMEM : DOCK_E_DEVICE, "%s: %s", what,
              hipGetErrorString(e));
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct WsLayout {
  size_t small, keys, order, bucket, status, kstar, cs, item_orient, item_align, total;
};

WsLayout ws_layout(int64_t L, int64_t total_rot, int O, int S, int passes, int n_align) {
  WsLayout w;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  w.small = take(sizeof(int32_t) * kSmallInts);
  w.keys = take(sizeof(unsigned long long) * (size_t)L);
  w.order = take(sizeof(int32_t) * (size_t)L);
  w.bucket = take(sizeof(int32_t) * (size_t)L);
  w.status = take(sizeof(int32_t) * (size_t)L);
  w.kstar = take(sizeof(int16_t) * (size_t)total_rot * (size_t)passes * (size_t)O);
  w.cs = take(sizeof(float2) * (size_t)S);
  // alignment: one rigid transform and one rotation index per item
  w.item_orient = n_align > 0 ? take(sizeof(float) * 12 * (size_t)L * (size_t)O) : 0;
  w.item_align = n_align > 0 ? take(sizeof(int16_t) * (size_t)L * (size_t)O) : 0;
  w.total = off;
  return w;
}

int grow(void **buf, size_t *have, size_t need) {
  if (*have >= need && *buf) return DOCK_OK;
  if (*buf) (void)hipFree(*buf);
  *buf = nullptr;
  *have = 0;
  hipError_t e = hipMalloc(buf, need < kAlign ? kAlign : need);
  if (e != hipSuccess) {
    *buf = nullptr;
    return hip_fail(e, "hipMalloc(workspace)");
  }
  *have = need;
  return DOCK_OK;
}

int check_params(const dock_params *prm, int n_orient, int S) {
  if (!prm) return fail(DOCK_E_INVAL, "params is NULL");
  if (n_orient < 1) return fail(DOCK_E_INVAL, "n_orient must be >= 1");
  if (S < 1 || S > DOCK_MAX_STEPS) return fail(DOCK_E_LIMIT, "angle_steps %d outside [1, %d]", S, DOCK_MAX_STEPS);
  if (!(prm->r_bump >= 0.0f) || !std::isfinite(prm->r_bump))
    return fail(DOCK_E_INVAL, "r_bump must be finite and >= 0");
  if (prm->passes < 1 || prm->passes > DOCK_MAX_PASSES)
    return fail(DOCK_E_LIMIT, "passes %d outside [1, %d]", prm->passes, DOCK_MAX_PASSES);
  if (prm->mode != DOCK_MODE_PLAIN && prm->mode != DOCK_MODE_LEARNED)
    return fail(DOCK_E_INVAL, "unknown mode %d", prm->mode);
  if (prm->max_atoms < 0 || prm->max_atoms > DOCK_MAX_ATOMS)
    return fail(DOCK_E_LIMIT, "max_atoms %d outside [0, %d]", prm->max_atoms, DOCK_MAX_ATOMS);
  if (prm->n_align < 0 || prm->n_align > DOCK_MAX_ALIGN)
    return fail(DOCK_E_LIMIT, "n_align %d outside [0, %d]", prm->n_align, DOCK_MAX_ALIGN);
  if (prm->n_align > 0 && !prm->align_rot) return fail(DOCK_E_INVAL, "align_rot is NULL");
  return DOCK_OK;
}

// Host check of an alignment set: finite, orthonormal rows within 1e-3.
int check_rotations_host(const float *rot, int n) {
  for (int a = 0; a < n; ++a) {
    const float *m = rot + 9 * (size_t)a;
    for (int k = 0; k < 9; ++k)
      if (!std::isfinite(m[k])) return fail(DOCK_E_INVAL, "alignment rotation %d is not finite", a);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double d = (double)m[3 * i] * m[3 * j] + (double)m[3 * i + 1] * m[3 * j + 1] +
                   (double)m[3 * i + 2] * m[3 * j + 2];
        if (std::fabs(d - (i == j ? 1.0 : 0.0)) > 1e-3)
          return fail(DOCK_E_INVAL, "alignment matrix %d is not orthonormal", a);
      }
  }
  return DOCK_OK;
}

// Full host-side check of a CSR batch (synchronous path).
int check_ligands_host(const dock_ligands *L, int *max_n, int *max_r = nullptr) {
  if (!L) return fail(DOCK_E_INVAL, "ligands is NULL");
  if (L->n_ligands < 0) return fail(DOCK_E_INVAL, "n_ligands < 0");
  if (!L->atom_offset || !L->rot_offset) return fail(DOCK_E_INVAL, "offset array is NULL");
  const int nl = L->n_ligands;
  if (L->atom_offset[0] != 0 || L->rot_offset[0] != 0)
    return fail(DOCK_E_INVAL, "offsets must start at 0");
  if (L->atom_offset[nl] != L->total_atoms || L->rot_offset[nl] != L->total_rot)
    return fail(DOCK_E_INVAL, "total_atoms/total_rot do not match the offsets");
  if (L->total_rot > 0 && (!L->rot_axis || !L->move_offset))
    return fail(DOCK_E_INVAL, "rot_axis/move_offset is NULL");
  if (L->total_atoms > 0 && !L->xyz) return fail(DOCK_E_INVAL, "xyz is NULL");
  if (L->total_rot > 0) {
    if (L->move_offset[0] != 0 || L->move_offset[L->total_rot] != L->total_move)
      return fail(DOCK_E_INVAL, "move_offset must run from 0 to total_move");
    if (L->total_move > 0 && !L->move_atoms) return fail(DOCK_E_INVAL, "move_atoms is NULL");
  }
  int mx = 0, mr = 0;
  for (int l = 0; l < nl; ++l) {
    int n = L->atom_offset[l + 1] - L->atom_offset[l];
    int R = L->rot_offset[l + 1] - L->rot_offset[l];
    if (n < 1) return fail(DOCK_E_INVAL, "ligand %d has %d atoms", l, n);
    if (R < 0) return fail(DOCK_E_INVAL, "ligand %d: rot_offset decreases", l);
    if (n > DOCK_MAX_ATOMS) return fail(DOCK_E_LIMIT, "ligand %d has %d atoms (max %d)", l, n, DOCK_MAX_ATOMS);
    if (R > DOCK_MAX_ROT) return fail(DOCK_E_LIMIT, "ligand %d has %d rotamers (max %d)", l, R, DOCK_MAX_ROT);
    mx = n > mx ? n : mx;
    mr = R > mr ? R : mr;
    for (int r = L->rot_offset[l]; r < L->rot_offset[l + 1]; ++r) {
      int a = L->rot_axis[2 * r], b = L->rot_axis[2 * r + 1];
      if (a < 0 || a >= n || b < 0 || b >= n || a == b)
        return fail(DOCK_E_INVAL, "ligand %d rotamer %d: bad axis (%d, %d)", l, r, a, b);
      int m0 = L->move_offset[r], m1 = L->move_offset[r + 1];
      if (m1 < m0 || m1 - m0 > n - 2)
        return fail(DOCK_E_INVAL, "ligand %d rotamer %d: bad moving-set size", l, r);
      int prev = -1;
      for (int t = m0; t < m1; ++t) {
        int i = L->move_atoms[t];
        if (i <= prev || i >= n || i == a || i == b)
          return fail(DOCK_E_INVAL, "ligand %d rotamer %d: bad moving atom %d", l, r, i);
        prev = i;
      }
    }
  }
  *max_n = mx;
  if (max_r) *max_r = mr;
  return DOCK_OK;
}

int maxn_bucket(int max_atoms) { return max_atoms <= 64 ? 64 : (max_atoms <= 128 ? 128 : 256); }

void free_learned(dock_pocket *p) {
  for (void *q : {(void *)p->lw_pose, (void *)p->lw_feat, (void *)p->lw_valid, (void *)p->lw_z[0],
                  (void *)p->lw_z[1], (void *)p->lw_z[2], (void *)p->lw_z[3], (void *)p->lw_a[0],
                  (void *)p->lw_a[1], (void *)p->lw_a[2]})
    if (q) (void)hipFree(q);
  p->lw_pose = nullptr;
  p->lw_feat = nullptr;
  p->lw_valid = nullptr;
  for (auto &z : p->lw_z) z = nullptr;
  for (auto &a : p->lw_a) a = nullptr;
  p->lw_items = p->lw_rows = 0;
  p->lw_nmax = p->lw_tiles = 0;
}

int grow_learned(dock_pocket *p, int64_t items, int nmax, int tiles) {
  const int64_t rows = (items + 63) / 64 * 64;
  if (items <= p->lw_items && nmax <= p->lw_nmax && tiles <= p->lw_tiles && p->lw_pose)
    return DOCK_OK;
  free_learned(p);
  hipError_t e = hipSuccess;
  auto A = [&](void **q, size_t b) {
    if (e == hipSuccess) e = hipMalloc(q, b < 256 ? 256 : b);
  };
  A((void **)&p->lw_pose, sizeof(float4) * (size_t)items * nmax);
  A((void **)&p->lw_feat, sizeof(uint16_t) * (size_t)rows * 64);
  A((void **)&p->lw_valid, sizeof(uint64_t) * (size_t)items * tiles);
  for (auto &z : p->lw_z) A((void **)&z, sizeof(float) * (size_t)rows * 256);
  for (auto &a : p->lw_a) A((void **)&a, sizeof(uint16_t) * (size_t)rows * 256);
  // padding rows of the feature matrix stay zero
  if (e == hipSuccess) e = hipMemset(p->lw_feat, 0, sizeof(uint16_t) * (size_t)rows * 64);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    free_learned(p);
    return hip_fail(e, "learned-mode buffers");
  }
  p->lw_items = items;
  p->lw_rows = rows;
  p->lw_nmax = nmax;
  p->lw_tiles = tiles;
  return DOCK_OK;
}

// max_rot: the most rotamers a ligand of this batch has (synchronous calls
// know it exactly, asynchronous ones take dock_params.max_rot, 0 meaning
// 255); in learned mode the step launches cover max_rot x passes steps and
// the device validation rejects ligands with more rotamers (DOCK_E_LIMIT).
int enqueue_batch(dock_pocket *p, const dock_ligands *ligs, const float *orient, int O, int S,
                  const dock_params *prm, const dock_results *out, void *ws, size_t ws_bytes,
                  hipStream_t st, int max_rot, uint16_t *emit_x = nullptr,
                  uint16_t *emit_t = nullptr, uint32_t *emit_mask = nullptr,
                  bool events = true) {
  const int64_t L = ligs->n_ligands;
  const int max_atoms = prm->max_atoms > 0 ? prm->max_atoms : DOCK_MAX_ATOMS;
  if (L * (int64_t)O >= ((int64_t)1 << 31)) return fail(DOCK_E_LIMIT, "n_ligands * n_orient >= 2^31");
  const bool learned = prm->mode == DOCK_MODE_LEARNED;
  if (learned) {
    if (!p->prop_wb) return fail(DOCK_E_STATE, "no learned proposal loaded (dock_load_proposal)");
    if (prm->top_k < 1 || prm->top_k > 63) return fail(DOCK_E_LIMIT, "top_k outside [1, 63]");
    if (prm->top_k * ((S + 255) / 256) + 1 > 512)
      return fail(DOCK_E_LIMIT, "top_k x ceil(angle_steps / 256) must be below 512");
  }
  if (max_rot < 0 || max_rot > DOCK_MAX_ROT) return fail(DOCK_E_LIMIT, "max_rot outside [0, 255]");
  WsLayout w = ws_layout(L, ligs->total_rot, O, S, prm->passes, prm->n_align);
  if (ws_bytes < w.total) return fail(DOCK_E_INVAL, "workspace too small: %zu < %zu", ws_bytes, w.total);
  char *base = (char *)ws;
  SweepArgs A{};
  A.grid = p->view;
  A.lig = LigView{ligs->n_ligands, ligs->total_atoms, ligs->total_rot, ligs->total_move,
                  ligs->atom_offset, ligs->xyz, ligs->rot_offset, ligs->rot_axis,
                  ligs->move_offset, ligs->move_atoms};
  A.orient = orient;
  A.n_orient = O;
  A.orient_stride = 0;
  A.S = S;
  A.passes = prm->passes;
  A.r2 = prm->r_bump * prm->r_bump;
  A.cs = (const float2 *)(base + w.cs);
  A.order = (const int32_t *)(base + w.order);
  A.status = out->status ? out->status : (const int32_t *)(base + w.status);
  A.small = (int32_t *)(base + w.small);
  A.queue = A.small;
  A.n_items = (int32_t)(L * O);
  A.claim = p->plan.items_per_claim;
  const bool timed = (prm->flags & DOCK_FLAG_TIME_SWEEP) != 0;
  // Timing events bracket the kernels only in eager calls: recorded inside a
  // captured graph they do not, so a graph is timed around its launch.
  const bool ev = timed && events;
  A.work = timed ? (unsigned long long *)(A.small + 4) : nullptr;
  A.keys = (unsigned long long *)(base + w.keys);
  A.kstar = (int16_t *)(base + w.kstar);
  A.all_scores = out->all_scores;
  A.emit_x = emit_x;
  A.emit_t = emit_t;
  A.emit_mask = emit_mask;
  int32_t *counts = A.small + 64, *cursor = A.small + 64 + kSortBuckets;
  bool lpt = !(prm->flags & DOCK_FLAG_NO_LPT) && !learned;
  // size classes for the grouped mappings: plain pruned sweeps in LPT order
  LaunchPlan plan = p->plan;
  if (!lpt || emit_x || (prm->flags & DOCK_FLAG_DIRECT_BUMP) || S > DOCK_GROUP_MAX_STEPS)
    plan.group16_atoms = plan.group32_atoms = 0;
  const int c16 = min(plan.group16_atoms, max_atoms);
  const int c32 = max(c16, min(plan.group32_atoms, max_atoms));
  const int split = c32 > c16 ? plan.group32_split : 0;
  hipError_t e = enqueue_prepare(A, max_atoms, learned ? max_rot : DOCK_MAX_ROT, lpt, c16, split,
                                 c32, (int32_t *)(base + w.bucket), counts, cursor,
                                 A.small + 1, st);
  if (e != hipSuccess) return hip_fail(e, "prepare kernels");
  const int maxn = maxn_bucket(max_atoms);
  // rigid alignment: per-item transforms replace the shared orientation table
  const int16_t *item_align = nullptr;
  if (prm->n_align > 0 && L > 0) {
    AlignArgs AA{};
    AA.grid = p->view;
    AA.lig = A.lig;
    AA.orient = orient;
    AA.n_orient = O;
    AA.rot = prm->align_rot;
    AA.n_align = prm->n_align;
    AA.status = A.status;
    AA.item_orient = (float *)(base + w.item_orient);
    AA.item_align = (int16_t *)(base + w.item_align);
    if (ev && (e = hipEventRecord(p->ev_align[0], st)) != hipSuccess)
      return hip_fail(e, "hipEventRecord");
    if ((e = enqueue_align(AA, maxn, st)) != hipSuccess) return hip_fail(e, "alignment kernel");
    if (ev) {
      if ((e = hipEventRecord(p->ev_align[1], st)) != hipSuccess) return hip_fail(e, "hipEventRecord");
      p->align_timed = true;
    }
    if (out->all_align_idx &&
        (e = hipMemcpyAsync(out->all_align_idx, AA.item_align, sizeof(int16_t) * (size_t)L * O,
                            hipMemcpyDeviceToDevice, st)) != hipSuccess)
      return hip_fail(e, "copy all_align_idx");
    A.orient = AA.item_orient;
    A.orient_stride = O;
    item_align = AA.item_align;
  }
  if (learned) {
    const int nmax = (max_atoms + 15) / 16 * 16;
    int rc = grow_learned(p, L * O, nmax, (S + 63) / 64);
    if (rc) return rc;
    int32_t *nfb = out->n_fallback;
    if (!nfb) {
      if (p->lw_fallback_n < L) {
        if (p->lw_fallback) (void)hipFree(p->lw_fallback);
        p->lw_fallback = nullptr;
        p->lw_fallback_n = 0;
        if ((e = hipMalloc((void **)&p->lw_fallback, sizeof(int32_t) * (L > 0 ? L : 1))) != hipSuccess)
          return hip_fail(e, "hipMalloc(n_fallback)");
        p->lw_fallback_n = L;
      }
      nfb = p->lw_fallback;
    }
    if ((e = enqueue_fill_i32(nfb, (int)L, 0, st)) != hipSuccess) return hip_fail(e, "fill");
    LearnedArgs LA{};
    LA.sw = A;
    LA.nmax = nmax;
    LA.pose = p->lw_pose;
    LA.feat = p->lw_feat;
    LA.valid = p->lw_valid;
    LA.pred = p->lw_z[3];
    LA.tiles = (S + 63) / 64;
    LA.top_k = prm->top_k;
    LA.margin = prm->margin;
    LA.n_fallback = nfb;
    if (ev && (e = hipEventRecord(p->ev_ring[p->ring_next][0], st)) != hipSuccess)
      return hip_fail(e, "hipEventRecord");
    if ((e = enqueue_learned_begin(LA, p->n_cu, st)) != hipSuccess)
      return hip_fail(e, "learned begin kernel");
    const int steps = max_rot * prm->passes;
    const int rows = (int)((L * O + 63) / 64 * 64);
    for (int s = 0; s < steps; ++s) {
      e = mlp_infer(p->lw_feat, rows, p->prop_wb, p->prop_w, p->lw_z[3], st);
      if (e == hipSuccess) e = enqueue_learned_step(LA, s, p->n_cu, st);
      if (e != hipSuccess) return hip_fail(e, "learned step");
    }
    if (timed) {
      if (ev && (e = hipEventRecord(p->ev_ring[p->ring_next][1], st)) != hipSuccess)
        return hip_fail(e, "hipEventRecord");
      e = hipMemcpyAsync(p->h_work, A.small + 4, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st);
      if (e == hipSuccess && ev) e = hipEventRecord(p->ev_work, st);
      if (e != hipSuccess) return hip_fail(e, "timing");
      if (ev) ring_advance(p);
    }
    FinalOut F{out->best_score, out->best_orient, out->angle_idx, out->xyz_out, out->align_idx,
               item_align};
    e = enqueue_finalize(A, F, maxn, kSweepPruned, st);
    if (e != hipSuccess) return hip_fail(e, "finalize kernel");
    if (out->all_angle_idx && ligs->total_rot > 0) {
      e = hipMemcpyAsync(out->all_angle_idx, A.kstar,
                         sizeof(int16_t) * (size_t)ligs->total_rot * prm->passes * O,
                         hipMemcpyDeviceToDevice, st);
      if (e != hipSuccess) return hip_fail(e, "copy all_angle_idx");
    }
    return DOCK_OK;
  }
  if (ev && (e = hipEventRecord(p->ev_ring[p->ring_next][0], st)) != hipSuccess)
    return hip_fail(e, "hipEventRecord");
  const SweepMode mode = (prm->flags & DOCK_FLAG_DIRECT_BUMP) ? kSweepDirect : kSweepPruned;
  if (mode == kSweepDirect)
    e = enqueue_sweep(A, maxn, p->plan, p->n_cu, st);
  else
    e = enqueue_sweep_pruned(A, max_atoms, plan, p->n_cu, st);
  if (e != hipSuccess) return hip_fail(e, "sweep kernel");
  if (timed) {
    if (ev && (e = hipEventRecord(p->ev_ring[p->ring_next][1], st)) != hipSuccess)
      return hip_fail(e, "hipEventRecord");
    e = hipMemcpyAsync(p->h_work, A.small + 4, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return hip_fail(e, "copy pair count");
    if (ev && (e = hipEventRecord(p->ev_work, st)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    if (ev) ring_advance(p);
  }
  FinalOut F{out->best_score, out->best_orient, out->angle_idx, out->xyz_out, out->align_idx,
             item_align};
  e = enqueue_finalize(A, F, maxn, mode, st);
  if (e != hipSuccess) return hip_fail(e, "finalize kernel");
  if (out->all_angle_idx && ligs->total_rot > 0) {
    e = hipMemcpyAsync(out->all_angle_idx, A.kstar,
                       sizeof(int16_t) * (size_t)ligs->total_rot * prm->passes * O,
                       hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "copy all_angle_idx");
  }
  return DOCK_OK;
}

}  // namespace

namespace dock {

int abi_check_sync(const dock_ligands *ligs, const float *orient, int n_orient, int angle_steps,
                   const dock_params *prm, int *max_n, int *max_r) {
  int rc = check_params(prm, n_orient, angle_steps);
  if (rc) return rc;
  rc = check_ligands_host(ligs, max_n, max_r);
  if (rc) return rc;
  for (int a = 0; a < n_orient * 12; ++a)
    if (!std::isfinite(orient[a])) return fail(DOCK_E_INVAL, "orientation table is not finite");
  if (prm->n_align > 0 && (rc = check_rotations_host(prm->align_rot, prm->n_align)) != DOCK_OK)
    return rc;
  for (int64_t a = 0; a < ligs->total_atoms * 3; ++a)
    if (!std::isfinite(ligs->xyz[a])) return fail(DOCK_E_INVAL, "coordinates are not finite");
  return DOCK_OK;
}

int abi_enqueue_plain(dock_pocket *p, const dock_ligands *ligs, const float *orient, int n_orient,
                      int angle_steps, const dock_params *prm, const dock_results *out, void *ws,
                      size_t ws_bytes, hipStream_t st) {
  if (prm->mode != DOCK_MODE_PLAIN) return fail(DOCK_E_INVAL, "plain mode expected");
  return enqueue_batch(p, ligs, orient, n_orient, angle_steps, prm, out, ws, ws_bytes, st,
                       DOCK_MAX_ROT);
}

int abi_device(const dock_pocket *p) { return p->device; }

int abi_host_grid(dock_pocket *p, HostGrid *g) {
  const size_t nvox = (size_t)p->view.nx * p->view.ny * p->view.nz;
  if (p->host_grid.size() != nvox) {
    try {
      p->host_grid.resize(nvox);
    } catch (const std::bad_alloc &) {
      return fail(DOCK_E_NOMEM, "host copy of the grid");
    }
    hipError_t e = hipMemcpy(p->host_grid.data(), p->d_grid, sizeof(float) * nvox, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      p->host_grid.clear();
      return hip_fail(e, "grid download");
    }
  }
  *g = HostGrid{p->host_grid.data(), p->view.nx, p->view.ny, p->view.nz, p->view.ox, p->view.oy,
                p->view.oz, p->view.inv_h};
  return DOCK_OK;
}

HybridCache *abi_hybrid_cache(dock_pocket *p) { return &p->hybrid; }

void abi_lock(dock_pocket *p) { p->mu.lock(); }
void abi_unlock(dock_pocket *p) { p->mu.unlock(); }

}  // namespace dock

extern "C" {

const char *dock_strerror(int code) {
  switch (code) {
    case DOCK_OK: return "ok";
    case DOCK_E_INVAL: return "invalid argument";
    case DOCK_E_LIMIT: return "outside a documented limit";
    case DOCK_E_NOMEM: return "out of memory";
    case DOCK_E_DEVICE: return "HIP device error";
    case DOCK_E_CANCELLED: return "cancelled";
    case DOCK_E_STATE: return "invalid state";
    default: return "unknown error";
  }
}

const char *dock_last_error(void) { return g_last_error.c_str(); }

int dock_last_sweep_work(dock_pocket *p, uint64_t *kept_pairs, uint64_t *atom_angle_evals) {
  g_last_error.clear();
  if (!p || !kept_pairs || !atom_angle_evals) return fail(DOCK_E_INVAL, "NULL argument");
  if (p->ring_count == 0) return fail(DOCK_E_STATE, "no call with DOCK_FLAG_TIME_SWEEP yet");
  DeviceGuard g(p->device);
  hipError_t e = hipEventSynchronize(p->ev_work);
  if (e != hipSuccess) return hip_fail(e, "sweep counters");
  *kept_pairs = (uint64_t)((volatile unsigned long long *)p->h_work)[0];
  *atom_angle_evals = (uint64_t)((volatile unsigned long long *)p->h_work)[1];
  return DOCK_OK;
}

int dock_set_launch(dock_pocket *p, int waves_per_block, int blocks_per_cu,
                    int items_per_claim) {
  g_last_error.clear();
  if (!p) return fail(DOCK_E_INVAL, "NULL pocket");
  if (waves_per_block != 0 && waves_per_block != 1 && waves_per_block != 2 && waves_per_block != 4)
    return fail(DOCK_E_INVAL, "waves_per_block must be 0 (automatic), 1, 2 or 4");
  if (blocks_per_cu < 0) return fail(DOCK_E_INVAL, "blocks_per_cu must be >= 0");
  if (items_per_claim < 1 || items_per_claim > 64)
    return fail(DOCK_E_INVAL, "items_per_claim must be in [1, 64]");
  p->plan = LaunchPlan{waves_per_block, blocks_per_cu, items_per_claim, p->plan.group16_atoms,
                       p->plan.group32_atoms, p->plan.group32_split};
  return DOCK_OK;
}

int dock_set_group_mapping(dock_pocket *p, int atoms16, int atoms32) {
  g_last_error.clear();
  if (!p) return fail(DOCK_E_INVAL, "NULL pocket");
  if (atoms16 < 0 || atoms16 > kGroupMaxAtoms16 || atoms32 < 0 || atoms32 > kGroupMaxAtoms32)
    return fail(DOCK_E_LIMIT, "group bounds (%d, %d) outside [0, %d] x [0, %d]", atoms16, atoms32,
                kGroupMaxAtoms16, kGroupMaxAtoms32);
  if (atoms32 != 0 && atoms32 <= atoms16)
    return fail(DOCK_E_INVAL, "the 32-lane class must hold larger ligands than the 16-lane class");
  p->plan.group16_atoms = atoms16;
  p->plan.group32_atoms = atoms32;
  return DOCK_OK;
}

int dock_set_group_split(dock_pocket *p, int atoms) {
  g_last_error.clear();
  if (!p) return fail(DOCK_E_INVAL, "NULL pocket");
  if (atoms != 0 && (atoms < kGroupSplitMin || atoms > kGroupMaxAtoms32))
    return fail(DOCK_E_LIMIT, "group split %d: 0 or within [%d, %d]", atoms, kGroupSplitMin,
                kGroupMaxAtoms32);
  p->plan.group32_split = atoms;
  return DOCK_OK;
}

int dock_get_group_split(dock_pocket *p, int *atoms) {
  g_last_error.clear();
  if (!p || !atoms) return fail(DOCK_E_INVAL, "NULL argument");
  *atoms = p->plan.group32_split;
  return DOCK_OK;
}

int dock_get_group_mapping(dock_pocket *p, int *atoms16, int *atoms32) {
  g_last_error.clear();
  if (!p || !atoms16 || !atoms32) return fail(DOCK_E_INVAL, "NULL argument");
  *atoms16 = p->plan.group16_atoms;
  *atoms32 = p->plan.group32_atoms;
  return DOCK_OK;
}

int dock_get_launch(dock_pocket *p, int *waves_per_block, int *blocks_per_cu,
                    int *items_per_claim) {
  g_last_error.clear();
  if (!p || !waves_per_block || !blocks_per_cu || !items_per_claim)
    return fail(DOCK_E_INVAL, "NULL argument");
  *waves_per_block = p->plan.waves_per_block;
  *blocks_per_cu = p->plan.blocks_per_cu;
  *items_per_claim = p->plan.items_per_claim;
  return DOCK_OK;
}

// Seeded subset of ligand indices (SplitMix64-driven partial shuffle).
static std::vector<int> sample_ligands(int n, int count, uint64_t seed) {
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  uint64_t st = seed;
  auto next = [&]() {
    uint64_t z = (st += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  if (count > n) count = n;
  for (int i = 0; i < count; ++i) {
    int j = i + (int)(next() % (uint64_t)(n - i));
    std::swap(idx[i], idx[j]);
  }
  idx.resize(count);
  std::sort(idx.begin(), idx.end());
  return idx;
}

int dock_autotune(dock_pocket *p, const dock_ligands *ligs, const float *orient, int n_orient,
                  int angle_steps, const dock_params *prm, int sample_ligands_n, uint64_t seed,
                  dock_tune_entry *entries, int max_entries, int *n_entries) {
  g_last_error.clear();
  if (!p || !ligs || !orient || !prm) return fail(DOCK_E_INVAL, "NULL argument");
  int rc = check_params(prm, n_orient, angle_steps);
  if (rc) return rc;
  int max_n = 0;
  rc = check_ligands_host(ligs, &max_n);
  if (rc) return rc;
  if (ligs->n_ligands < 1 || sample_ligands_n < 1)
    return fail(DOCK_E_INVAL, "autotune needs at least one ligand");
  // seeded sub-batch
  std::vector<int> pick = sample_ligands(ligs->n_ligands, sample_ligands_n, seed);
  std::vector<int32_t> ao{0}, ro{0}, ax, mo{0};
  std::vector<float> xyz;
  std::vector<int16_t> mv;
  for (int l : pick) {
    int a0 = ligs->atom_offset[l], a1 = ligs->atom_offset[l + 1];
    int r0 = ligs->rot_offset[l], r1 = ligs->rot_offset[l + 1];
    xyz.insert(xyz.end(), ligs->xyz + 3 * (size_t)a0, ligs->xyz + 3 * (size_t)a1);
    ao.push_back(ao.back() + (a1 - a0));
    for (int r = r0; r < r1; ++r) {
      ax.push_back(ligs->rot_axis[2 * r]);
      ax.push_back(ligs->rot_axis[2 * r + 1]);
      for (int t = ligs->move_offset[r]; t < ligs->move_offset[r + 1]; ++t)
        mv.push_back(ligs->move_atoms[t]);
      mo.push_back((int32_t)mv.size());
    }
    ro.push_back(ro.back() + (r1 - r0));
  }
  dock_ligands sub{(int32_t)pick.size(), ao.back(), ro.back(), (int64_t)mv.size(), ao.data(),
                   xyz.data(), ro.data(), ax.data(), mo.data(), mv.data()};
  const int64_t L = sub.n_ligands, NR = sub.total_rot, NA = sub.total_atoms;
  std::vector<float> bs(L), xo(3 * NA + 3);
  std::vector<int32_t> bo(L), stv(L);
  std::vector<int16_t> ai(NR * prm->passes + 1);
  dock_results res{bs.data(), bo.data(), ai.data(), xo.data(), nullptr, nullptr, stv.data(), nullptr};
  dock_params tp = *prm;
  tp.flags |= DOCK_FLAG_TIME_SWEEP;
  const int waves[] = {0, 1, 2, 4};  // 0: per class, the size with the most resident waves
  const int claims[] = {4, 16, 32, 64};
  // size classes docked in groups: none, four (16-lane, 32-lane) bounds, and
  // one with the 32-lane ligands in classes 32 atoms wide
  const int groups[][3] = {{0, 0, 0},    {48, 96, 0},  {64, 128, 0},
                           {80, 128, 0}, {80, 192, 0}, {64, 192, 32}};
  LaunchPlan best_plan = p->plan;
  float best_ms = 0.0f;
  int n = 0;
  for (const auto &gm : groups)
   for (int w : waves)
    for (int c : claims) {
      p->plan = LaunchPlan{w, 0, c, gm[0], gm[1], gm[2]};
      float ms_sum = 0.0f;
      for (int rep = 0; rep < 3; ++rep) {
        rc = dock_batch(p, &sub, orient, n_orient, angle_steps, &tp, &res);
        if (rc) {
          p->plan = best_plan;
          return rc;
        }
        float ms = 0.0f;
        rc = dock_last_sweep_ms(p, &ms);
        if (rc) return rc;
        if (rep > 0) ms_sum += ms;  // first run warms caches
      }
      const float ms = ms_sum / 2.0f;
      if (entries && n < max_entries) entries[n] = dock_tune_entry{w, 0, c, ms, gm[0], gm[1], gm[2]};
      ++n;
      if (best_ms == 0.0f || ms < best_ms) {
        best_ms = ms;
        best_plan = LaunchPlan{w, 0, c, gm[0], gm[1], gm[2]};
      }
    }
  p->plan = best_plan;
  if (n_entries) *n_entries = n < max_entries ? n : max_entries;
  return DOCK_OK;
}

int dock_last_sweep_ms(dock_pocket *p, float *ms) { return dock_sweep_ms_history(p, 1, ms); }

int dock_sweep_ms_history(dock_pocket *p, int n, float *ms) {
  g_last_error.clear();
  if (!p || !ms) return fail(DOCK_E_INVAL, "NULL argument");
  if (n < 1 || n > kTimingRing) return fail(DOCK_E_INVAL, "n outside [1, %d]", kTimingRing);
  if (p->ring_count < n)
    return fail(DOCK_E_STATE, "%d calls with DOCK_FLAG_TIME_SWEEP so far, %d asked for", p->ring_count, n);
  DeviceGuard g(p->device);
  hipError_t e = hipSuccess;
  for (int i = 0; i < n && e == hipSuccess; ++i) {
    const int slot = (p->ring_next - n + i + 2 * kTimingRing) % kTimingRing;  // oldest first
    e = hipEventSynchronize(p->ev_ring[slot][1]);
    if (e == hipSuccess) e = hipEventElapsedTime(ms + i, p->ev_ring[slot][0], p->ev_ring[slot][1]);
  }
  return e == hipSuccess ? DOCK_OK : hip_fail(e, "sweep timing");
}

size_t dock_workspace_size(int32_t n_ligands, int64_t total_rot, int n_orient, int angle_steps,
                           int passes, int n_align) {
  if (n_ligands < 0 || total_rot < 0 || n_orient < 1 || angle_steps < 1 || passes < 1 ||
      n_align < 0)
    return 0;
  return ws_layout(n_ligands, total_rot, n_orient, angle_steps, passes, n_align).total;
}

int dock_last_align_ms(dock_pocket *p, float *ms) {
  g_last_error.clear();
  if (!p || !ms) return fail(DOCK_E_INVAL, "NULL argument");
  if (!p->align_timed) return fail(DOCK_E_STATE, "no aligned call with DOCK_FLAG_TIME_SWEEP yet");
  DeviceGuard g(p->device);
  hipError_t e = hipEventSynchronize(p->ev_align[1]);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, p->ev_align[0], p->ev_align[1]);
  return e == hipSuccess ? DOCK_OK : hip_fail(e, "alignment timing");
}

int dock_init_pocket(const float *grid, int nx, int ny, int nz, const float origin[3],
                     float spacing, dock_pocket **out) {
  g_last_error.clear();
  if (!out) return fail(DOCK_E_INVAL, "out is NULL");
  *out = nullptr;
  if (!grid || !origin) return fail(DOCK_E_INVAL, "grid or origin is NULL");
  if (nx < 1 || ny < 1 || nz < 1 || nx > 4096 || ny > 4096 || nz > 4096)
    return fail(DOCK_E_LIMIT, "grid dims %d x %d x %d outside [1, 4096]", nx, ny, nz);
  if ((int64_t)nx * ny * nz >= ((int64_t)1 << 30))
    return fail(DOCK_E_LIMIT, "grid holds 2^30 voxels or more");
  if (!(spacing > 0.0f) || !std::isfinite(spacing)) return fail(DOCK_E_INVAL, "spacing must be > 0");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(origin[a])) return fail(DOCK_E_INVAL, "origin must be finite");
  dock_pocket *p = new (std::nothrow) dock_pocket;
  if (!p) return fail(DOCK_E_NOMEM, "host allocation");
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "hipGetDevice");
  }
  e = hipDeviceGetAttribute(&p->n_cu, hipDeviceAttributeMultiprocessorCount, p->device);
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "hipDeviceGetAttribute");
  }
  if (p->device < 0 || p->device >= kMaxDevices) {
    delete p;
    return fail(DOCK_E_LIMIT, "device ordinal %d outside [0, %d)", p->device, kMaxDevices);
  }
  {
    // once per device, with that device current (it is: p->device is the
    // current device)
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[p->device]) {
      void *ptr = nullptr;
      e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !ptr) {
        delete p;
        return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
      }
      g_scratch_ptr[p->device] = ptr;
    }
    p->scratch = g_scratch_ptr[p->device];
  }
  size_t bytes = sizeof(float) * (size_t)nx * ny * nz;
  e = hipMalloc((void **)&p->d_grid, bytes);
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "hipMalloc(grid)");
  }
  e = hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking);
  for (auto &pair : p->ev_ring)
    for (hipEvent_t &x : pair)
      if (e == hipSuccess) e = hipEventCreate(&x);
  if (e == hipSuccess) e = hipEventCreate(&p->ev_work);
  if (e == hipSuccess) e = hipEventCreate(&p->ev_align[0]);
  if (e == hipSuccess) e = hipEventCreate(&p->ev_align[1]);
  if (e == hipSuccess) e = hipHostMalloc((void **)&p->h_work, 2 * sizeof(unsigned long long), 0);
  if (e == hipSuccess) e = hipMemcpyAsync(p->d_grid, grid, bytes, hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) {
    int code = hip_fail(e, "grid upload");
    dock_free_pocket(p);
    return code;
  }
  p->view = GridView{p->d_grid, nx, ny, nz, origin[0], origin[1], origin[2], 1.0f / spacing};
  *out = p;
  return DOCK_OK;
}

void dock_free_pocket(dock_pocket *p) {
  if (!p) return;
  {
    DeviceGuard g(p->device);
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    if (p->d_grid) (void)hipFree(p->d_grid);
    if (p->ws) (void)hipFree(p->ws);
    if (p->io) (void)hipFree(p->io);
    if (p->sync_ws) (void)hipFree(p->sync_ws);
    if (p->stream) (void)hipStreamDestroy(p->stream);
    for (auto &pair : p->ev_ring)
      for (hipEvent_t x : pair)
        if (x) (void)hipEventDestroy(x);
    if (p->ev_work) (void)hipEventDestroy(p->ev_work);
    for (hipEvent_t ev : p->ev_align)
      if (ev) (void)hipEventDestroy(ev);
    if (p->h_work) (void)hipHostFree(p->h_work);
    if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    free_learned(p);
    if (p->hybrid.state && p->hybrid.release) p->hybrid.release(p->hybrid.state);
    if (p->lw_fallback) (void)hipFree(p->lw_fallback);
    if (p->prop_wb) (void)hipFree(p->prop_wb);
    if (p->prop_w) (void)hipFree(p->prop_w);
  }
  delete p;
}

}  // extern "C"

// Host-side checks shared by the two asynchronous entry points: sizes,
// non-NULL arrays and that every array is device-accessible.  Runs with the
// handle's device current.
static int check_async_args(const dock_pocket *p, const dock_ligands *ligs, const float *orient,
                            int n_orient, int angle_steps, const dock_params *prm,
                            const dock_results *out, const void *workspace) {
  if (!p || !ligs || !orient || !out) return fail(DOCK_E_INVAL, "NULL argument");
  int rc = check_params(prm, n_orient, angle_steps);
  if (rc) return rc;
  if (ligs->n_ligands < 0 || ligs->total_atoms < 0 || ligs->total_rot < 0 || ligs->total_move < 0)
    return fail(DOCK_E_INVAL, "negative size in ligands");
  if (ligs->n_ligands > 0 && (!ligs->atom_offset || !ligs->rot_offset || !ligs->xyz))
    return fail(DOCK_E_INVAL, "ligand array is NULL");
  if (ligs->total_rot > 0 && (!ligs->rot_axis || !ligs->move_offset))
    return fail(DOCK_E_INVAL, "rotamer array is NULL");
  if (ligs->total_move > 0 && !ligs->move_atoms) return fail(DOCK_E_INVAL, "move_atoms is NULL");
  if (ligs->n_ligands > 0 && (!out->best_score || !out->best_orient || !out->xyz_out))
    return fail(DOCK_E_INVAL, "result array is NULL");
  if (ligs->total_rot > 0 && !out->angle_idx) return fail(DOCK_E_INVAL, "angle_idx is NULL");
  {
    const bool rot = ligs->total_rot > 0, mv = ligs->total_move > 0, al = prm->n_align > 0;
    const std::pair<const void *, const char *> ptrs[] = {
        {ligs->atom_offset, "atom_offset"}, {ligs->xyz, "xyz"}, {ligs->rot_offset, "rot_offset"},
        {rot ? ligs->rot_axis : nullptr, "rot_axis"}, {rot ? ligs->move_offset : nullptr, "move_offset"},
        {mv ? ligs->move_atoms : nullptr, "move_atoms"}, {orient, "orient"},
        {al ? prm->align_rot : nullptr, "align_rot"}, {out->best_score, "best_score"},
        {out->best_orient, "best_orient"}, {rot ? out->angle_idx : nullptr, "angle_idx"},
        {out->xyz_out, "xyz_out"}, {out->all_scores, "all_scores"},
        {out->all_angle_idx, "all_angle_idx"}, {out->status, "status"},
        {out->n_fallback, "n_fallback"}, {out->align_idx, "align_idx"},
        {al ? out->all_align_idx : nullptr, "all_align_idx"}, {workspace, "workspace"}};
    if (ligs->n_ligands > 0)
      for (const auto &q : ptrs)
        if ((rc = abi_check_device(q.first, q.second)) != DOCK_OK) return rc;
  }
  if (prm->max_rot < 0 || prm->max_rot > DOCK_MAX_ROT)
    return fail(DOCK_E_LIMIT, "max_rot outside [0, 255]");
  return DOCK_OK;
}

extern "C" {

int dock_batch_async(dock_pocket *p, const dock_ligands *ligs, const float *orient, int n_orient,
                     int angle_steps, const dock_params *prm, dock_results *out, void *workspace,
                     size_t workspace_bytes, void *stream) {
  g_last_error.clear();
  if (!p) return fail(DOCK_E_INVAL, "NULL argument");
  DeviceGuard g(p->device);
  int rc = check_async_args(p, ligs, orient, n_orient, angle_steps, prm, out, workspace);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(p->mu);
  if (!workspace) {
    size_t need = dock_workspace_size(ligs->n_ligands, ligs->total_rot, n_orient, angle_steps,
                                      prm->passes, prm->n_align);
    rc = grow(&p->ws, &p->ws_bytes, need);
    if (rc) return rc;
    workspace = p->ws;
    workspace_bytes = p->ws_bytes;
  }
  hipStream_t st = (hipStream_t)stream;
  const int max_rot = prm->max_rot > 0 ? prm->max_rot : DOCK_MAX_ROT;
  if (!(prm->flags & DOCK_FLAG_GRAPH))
    return enqueue_batch(p, ligs, orient, n_orient, angle_steps, prm, out, workspace,
                         workspace_bytes, st, max_rot);
  if (!st) return fail(DOCK_E_INVAL, "DOCK_FLAG_GRAPH needs a non-default stream");
  // learned mode grows handle-owned buffers with allocations that a capture
  // cannot hold, and a graph would keep their addresses past a regrowth
  if (prm->mode == DOCK_MODE_LEARNED)
    return fail(DOCK_E_INVAL, "DOCK_FLAG_GRAPH cannot be combined with DOCK_MODE_LEARNED");
  // The launch sequence depends only on these values: replay it if they repeat.
  std::vector<unsigned char> key;
  auto put = [&](const void *v, size_t bytes) {
    key.insert(key.end(), (const unsigned char *)v, (const unsigned char *)v + bytes);
  };
  put(ligs, sizeof *ligs);
  put(&orient, sizeof orient);
  put(&n_orient, sizeof n_orient);
  put(&angle_steps, sizeof angle_steps);
  put(prm, sizeof *prm);
  put(out, sizeof *out);
  put(&workspace, sizeof workspace);
  put(&workspace_bytes, sizeof workspace_bytes);
  put(&p->plan, sizeof p->plan);
  hipError_t e;
  if (!p->graph_exec || key != p->graph_key) {
    if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->graph_exec = nullptr;
    p->graph = nullptr;
    p->graph_key.clear();
    if ((e = hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed)) != hipSuccess)
      return hip_fail(e, "hipStreamBeginCapture");
    rc = enqueue_batch(p, ligs, orient, n_orient, angle_steps, prm, out, workspace,
                       workspace_bytes, st, max_rot, nullptr, nullptr, nullptr, false);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(st, &graph);
    if (rc) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    if ((e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0)) != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return hip_fail(e, "hipGraphInstantiate");
    }
    p->graph = graph;
    p->graph_exec = exec;
    p->graph_key = key;
  }
  const bool timed = (prm->flags & DOCK_FLAG_TIME_SWEEP) != 0;
  if (timed && (e = hipEventRecord(p->ev_ring[p->ring_next][0], st)) != hipSuccess)
    return hip_fail(e, "hipEventRecord");
  if ((e = hipGraphLaunch(p->graph_exec, st)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  if (timed) {
    if ((e = hipEventRecord(p->ev_ring[p->ring_next][1], st)) != hipSuccess ||
        (e = hipEventRecord(p->ev_work, st)) != hipSuccess)
      return hip_fail(e, "hipEventRecord");
    ring_advance(p);
  }
  return DOCK_OK;
}

int dock_batch_async_static(dock_pocket *p, const dock_ligands *ligs, const float *orient,
                            int n_orient, int angle_steps, const dock_params *prm,
                            dock_results *out, void *stream) {
  g_last_error.clear();
  if (!p) return fail(DOCK_E_INVAL, "NULL argument");
  DeviceGuard g(p->device);
  int rc = check_async_args(p, ligs, orient, n_orient, angle_steps, prm, out, nullptr);
  if (rc) return rc;
  // learned mode grows handle-owned buffers and a graph needs instantiating:
  // both allocate
  if (prm->mode != DOCK_MODE_PLAIN)
    return fail(DOCK_E_INVAL, "dock_batch_async_static runs the plain sweep only");
  if (prm->flags & DOCK_FLAG_GRAPH)
    return fail(DOCK_E_INVAL, "dock_batch_async_static does not take DOCK_FLAG_GRAPH");
  if (!p->scratch) return fail(DOCK_E_STATE, "static workspace not resolved for this handle");
  const size_t need = dock_workspace_size(ligs->n_ligands, ligs->total_rot, n_orient, angle_steps,
                                          prm->passes, prm->n_align);
  if (need == 0 || need > (size_t)DOCK_STATIC_SCRATCH_BYTES)
    return fail(DOCK_E_LIMIT, "batch needs %zu bytes of workspace; the static workspace holds %zu",
                need, (size_t)DOCK_STATIC_SCRATCH_BYTES);
  std::lock_guard<std::mutex> lk(p->mu);
  const int max_rot = prm->max_rot > 0 ? prm->max_rot : DOCK_MAX_ROT;
  return enqueue_batch(p, ligs, orient, n_orient, angle_steps, prm, out, p->scratch,
                       (size_t)DOCK_STATIC_SCRATCH_BYTES, (hipStream_t)stream, max_rot);
}

static int run_sync(dock_pocket *p, const dock_ligands *ligs, const float *orient, int n_orient,
                    int angle_steps, const dock_params *prm, dock_results *out,
                    uint16_t *emit_x, uint16_t *emit_t, uint32_t *emit_mask) {
  int rc = check_params(prm, n_orient, angle_steps);
  if (rc) return rc;
  int max_n = 0, max_r = 0;
  rc = check_ligands_host(ligs, &max_n, &max_r);
  if (rc) return rc;
  const int64_t L = ligs->n_ligands, NA = ligs->total_atoms, NR = ligs->total_rot,
                NM = ligs->total_move;
  const int passes = prm->passes;
  for (int a = 0; a < n_orient * 12; ++a)
    if (!std::isfinite(orient[a])) return fail(DOCK_E_INVAL, "orientation table is not finite");
  const int NAL = prm->n_align;
  if (NAL > 0 && (rc = check_rotations_host(prm->align_rot, NAL)) != DOCK_OK) return rc;
  for (int64_t a = 0; a < NA * 3; ++a)
    if (!std::isfinite(ligs->xyz[a])) return fail(DOCK_E_INVAL, "coordinates are not finite");
  if (L == 0) return DOCK_OK;

  // device staging: inputs then outputs, each 256-B aligned
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  const size_t o_ao = take(4 * (L + 1)), o_xyz = take(12 * NA), o_ro = take(4 * (L + 1)),
               o_ax = take(8 * NR), o_mo = take(4 * (NR + 1)), o_mv = take(2 * NM),
               o_or = take(48 * (size_t)n_orient), o_bs = take(4 * L), o_bo = take(4 * L),
               o_ai = take(2 * NR * passes), o_xo = take(12 * NA),
               o_as = out->all_scores ? take(4 * L * n_orient) : 0,
               o_aai = out->all_angle_idx ? take(2 * NR * passes * n_orient) : 0,
               o_st = take(4 * L), o_fb = take(4 * L), o_rot = take(36 * (size_t)NAL),
               o_ali = take(2 * L), o_aal = out->all_align_idx ? take(2 * L * n_orient) : 0;
  std::lock_guard<std::mutex> lk(p->mu);
  DeviceGuard g(p->device);
  rc = grow(&p->io, &p->io_bytes, off);
  if (rc) return rc;
  const size_t need_ws = dock_workspace_size((int32_t)L, NR, n_orient, angle_steps, passes, NAL);
  rc = grow(&p->sync_ws, &p->sync_ws_bytes, need_ws);
  if (rc) return rc;
  char *d = (char *)p->io;
  hipStream_t st = p->stream;
  hipError_t e = hipSuccess;
  auto h2d = [&](size_t at, const void *src, size_t bytes) {
    if (e == hipSuccess && bytes) e = hipMemcpyAsync(d + at, src, bytes, hipMemcpyHostToDevice, st);
  };
  h2d(o_ao, ligs->atom_offset, 4 * (L + 1));
  h2d(o_xyz, ligs->xyz, 12 * NA);
  h2d(o_ro, ligs->rot_offset, 4 * (L + 1));
  if (NR > 0) {
    h2d(o_ax, ligs->rot_axis, 8 * NR);
    h2d(o_mo, ligs->move_offset, 4 * (NR + 1));
  }
  if (NM > 0) h2d(o_mv, ligs->move_atoms, 2 * NM);
  h2d(o_or, orient, 48 * (size_t)n_orient);
  if (NAL > 0) h2d(o_rot, prm->align_rot, 36 * (size_t)NAL);
  if (e != hipSuccess) return hip_fail(e, "batch upload");
  dock_ligands dl = *ligs;
  dl.atom_offset = (const int32_t *)(d + o_ao);
  dl.xyz = (const float *)(d + o_xyz);
  dl.rot_offset = (const int32_t *)(d + o_ro);
  dl.rot_axis = NR > 0 ? (const int32_t *)(d + o_ax) : nullptr;
  dl.move_offset = NR > 0 ? (const int32_t *)(d + o_mo) : nullptr;
  dl.move_atoms = NM > 0 ? (const int16_t *)(d + o_mv) : nullptr;
  dock_results dr{};
  dr.best_score = (float *)(d + o_bs);
  dr.best_orient = (int32_t *)(d + o_bo);
  dr.angle_idx = NR > 0 ? (int16_t *)(d + o_ai) : nullptr;
  dr.xyz_out = (float *)(d + o_xo);
  dr.all_scores = out->all_scores ? (float *)(d + o_as) : nullptr;
  dr.all_angle_idx = out->all_angle_idx ? (int16_t *)(d + o_aai) : nullptr;
  dr.status = (int32_t *)(d + o_st);
  dr.n_fallback = (int32_t *)(d + o_fb);
  dr.align_idx = out->align_idx ? (int16_t *)(d + o_ali) : nullptr;
  dr.all_align_idx = out->all_align_idx && NAL > 0 ? (int16_t *)(d + o_aal) : nullptr;
  dock_params pr = *prm;
  pr.max_atoms = max_n;
  pr.max_rot = max_r;
  pr.align_rot = NAL > 0 ? (const float *)(d + o_rot) : nullptr;
  rc = enqueue_batch(p, &dl, (const float *)(d + o_or), n_orient, angle_steps, &pr, &dr,
                     p->sync_ws, p->sync_ws_bytes, st, max_r, emit_x, emit_t, emit_mask);
  if (rc) return rc;
  auto d2h = [&](void *dst, size_t at, size_t bytes) {
    if (e == hipSuccess && dst && bytes)
      e = hipMemcpyAsync(dst, d + at, bytes, hipMemcpyDeviceToHost, st);
  };
  d2h(out->best_score, o_bs, 4 * L);
  d2h(out->best_orient, o_bo, 4 * L);
  if (NR > 0) d2h(out->angle_idx, o_ai, 2 * NR * passes);
  d2h(out->xyz_out, o_xo, 12 * NA);
  if (out->all_scores) d2h(out->all_scores, o_as, 4 * L * n_orient);
  if (out->all_angle_idx && NR > 0) d2h(out->all_angle_idx, o_aai, 2 * NR * passes * n_orient);
  d2h(out->status, o_st, 4 * L);
  d2h(out->align_idx, o_ali, 2 * L);
  if (NAL > 0) d2h(out->all_align_idx, o_aal, 2 * L * n_orient);
  if (prm->mode == DOCK_MODE_LEARNED) d2h(out->n_fallback, o_fb, 4 * L);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "batch run");
  return DOCK_OK;
}

int dock_batch(dock_pocket *p, const dock_ligands *ligs, const float *orient, int n_orient,
               int angle_steps, const dock_params *prm, dock_results *out) {
  g_last_error.clear();
  if (!p || !ligs || !orient || !out) return fail(DOCK_E_INVAL, "NULL argument");
  if (ligs->n_ligands > 0 && (!out->best_score || !out->best_orient || !out->xyz_out))
    return fail(DOCK_E_INVAL, "result array is NULL");
  if (ligs->total_rot > 0 && !out->angle_idx) return fail(DOCK_E_INVAL, "angle_idx is NULL");
  return run_sync(p, ligs, orient, n_orient, angle_steps, prm, out, nullptr, nullptr, nullptr);
}

int dock_emit_profiles(dock_pocket *p, const dock_ligands *ligs, const float *orient,
                       int n_orient, const dock_params *prm, uint16_t *x_out, uint16_t *t_out,
                       uint32_t *mask_out) {
  g_last_error.clear();
  if (!p || !ligs || !orient || !prm || !x_out || !t_out || !mask_out)
    return fail(DOCK_E_INVAL, "NULL argument");
  if (prm->mode != DOCK_MODE_PLAIN) return fail(DOCK_E_INVAL, "profiles come from the plain sweep");
  if (prm->n_align != 0) return fail(DOCK_E_INVAL, "profiles are emitted without alignment");
  {
    DeviceGuard g(p->device);
    int rc = abi_check_device(x_out, "x_out");
    if (rc == DOCK_OK) rc = abi_check_device(t_out, "t_out");
    if (rc == DOCK_OK) rc = abi_check_device(mask_out, "mask_out");
    if (rc) return rc;
  }
  dock_results none{};
  return run_sync(p, ligs, orient, n_orient, 256, prm, &none, x_out, t_out, mask_out);
}

int dock_load_proposal(dock_pocket *p, dock_mlp *m) {
  g_last_error.clear();
  if (!p || !m) return fail(DOCK_E_INVAL, "NULL argument");
  DeviceGuard g(p->device);
  std::lock_guard<std::mutex> lk(p->mu);
  hipError_t e = hipSuccess;
  if (!p->prop_wb) e = hipMalloc((void **)&p->prop_wb, sizeof(uint16_t) * kMlpParams);
  if (e == hipSuccess && !p->prop_w) e = hipMalloc((void **)&p->prop_w, sizeof(float) * kMlpParams);
  const uint16_t *wb = nullptr;
  const float *w = nullptr;
  mlp_export_weights(m, &wb, &w);
  if (e == hipSuccess)
    e = hipMemcpy(p->prop_wb, wb, sizeof(uint16_t) * kMlpParams, hipMemcpyDeviceToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->prop_w, w, sizeof(float) * kMlpParams, hipMemcpyDeviceToDevice);
  return e == hipSuccess ? DOCK_OK : hip_fail(e, "dock_load_proposal");
}

}  // extern "C"
