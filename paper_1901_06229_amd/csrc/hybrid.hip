// Hybrid host + GPU docking of one batch (paper §4.2: OpenMP threads and the
// accelerators work on one ligand queue, and §5.1: the CPU processes add to
// what the GPU process does).  MI355X-first form of that scheme:
//
//   * one dispenser hands out contiguous ranges of the batch: the GPU feeder
//     takes large ranges from the front (guided: a quarter of what is left,
//     between a quarter of the cap and the cap), host threads take a few
//     ligands at a time from the back, until the two ends meet;
//   * a GPU range is a contiguous slice of the caller's CSR arrays: packing
//     it is a few copies into pinned memory plus rebasing three offset
//     arrays, and its results come back as contiguous slices;
//   * the GPU feeder keeps two ranges in flight on two streams: while one
//     range's kernels run (the sweep sorts its own items by cost), the next is
//     packed and copied in, and the previous one's results are copied out
//     and written into the caller's arrays;
//   * host threads run the FP32 CPU sweep (cpu_sweep.cpp) on their ligands
//     and write their outputs directly.
// Every ligand is docked by exactly one side; both compute the same greedy
// sweep in FP32 (their results differ from each other only by rounding).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "abi_internal.h"
#include "cpu_sweep.h"
#include "dock.h"
#include "dock_internal.h"

namespace {

using dock::abi_fail;
using Clock = std::chrono::steady_clock;

int hip_err(hipError_t e, const char *what) {
  return abi_fail(e == hipErrorOutOfMemory ? DOCK_E_NOMEM : DOCK_E_DEVICE, "%s: %s", what,
                  hipGetErrorString(e));
}

constexpr size_t kAlign = 256;
size_t up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Ranges of the cost order handed to the two sides.
struct Dispenser {
  std::mutex mu;
  int64_t front = 0, back = 0;
  // [b, e) from the expensive end (GPU), at most n; false when empty
  bool take_front(int64_t n, int64_t *b, int64_t *e) {
    std::lock_guard<std::mutex> lk(mu);
    if (front >= back) return false;
    *b = front;
    *e = std::min(back, front + n);
    front = *e;
    return true;
  }
  // [b, e) from the cheap end (host threads)
  bool take_back(int64_t n, int64_t *b, int64_t *e) {
    std::lock_guard<std::mutex> lk(mu);
    if (front >= back) return false;
    *e = back;
    *b = std::max(front, back - n);
    back = *b;
    return true;
  }
};

// Section offsets of one packed chunk (inputs, then outputs), 256-B aligned.
struct ChunkLayout {
  int64_t L = 0, NA = 0, NR = 0, NM = 0;
  size_t ao, xyz, ro, ax, mo, mv, in_bytes;
  size_t bs, bo, ai, xo, as, aai, st, out_bytes;
  size_t ws_bytes;
  void plan(int64_t l, int64_t na, int64_t nr, int64_t nm, int O, int S, int passes, bool all) {
    L = l, NA = na, NR = nr, NM = nm;
    size_t off = 0;
    auto take = [&](size_t b) {
      const size_t at = off;
      off = up(off + b);
      return at;
    };
    ao = take(4 * (L + 1));
    xyz = take(12 * NA);
    ro = take(4 * (L + 1));
    ax = take(8 * NR);
    mo = take(4 * (NR + 1));
    mv = take(2 * NM);
    in_bytes = off;
    off = 0;
    bs = take(4 * L);
    bo = take(4 * L);
    ai = take(2 * NR * passes);
    xo = take(12 * NA);
    as = all ? take(4 * L * O) : 0;
    aai = all ? take(2 * NR * passes * O) : 0;
    st = take(4 * L);
    out_bytes = off;
    ws_bytes = dock_workspace_size((int32_t)L, NR, O, S, passes, 0);
  }
};

// One of the GPU feeder's two chunks in flight.
struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t ev_start = nullptr, ev_done = nullptr;
  char *h_in = nullptr, *h_out = nullptr;  // pinned
  char *d_in = nullptr, *d_out = nullptr, *d_ws = nullptr;
  size_t cap_in = 0, cap_out = 0, cap_ws = 0;
  bool busy = false;
  int64_t b = 0, e = 0;  // range of the cost order
  ChunkLayout lay;

  hipError_t grow(const ChunkLayout &c) {
    hipError_t err = hipSuccess;
    auto dev = [&](char **p, size_t *cap, size_t need) {
      if (err != hipSuccess || need <= *cap) return;
      if (*p) (void)hipFree(*p);
      *p = nullptr;
      *cap = 0;
      need = need * 5 / 4 + kAlign;
      err = hipMalloc((void **)p, need);
      if (err == hipSuccess) *cap = need;
    };
    auto host = [&](char **p, size_t need, size_t have) {
      if (err != hipSuccess || need <= have) return;
      if (*p) (void)hipHostFree(*p);
      *p = nullptr;
      err = hipHostMalloc((void **)p, need * 5 / 4 + kAlign, 0);
    };
    const size_t old_in = cap_in, old_out = cap_out;
    dev(&d_in, &cap_in, c.in_bytes);
    dev(&d_out, &cap_out, c.out_bytes);
    dev(&d_ws, &cap_ws, c.ws_bytes);
    host(&h_in, c.in_bytes, old_in);
    host(&h_out, c.out_bytes, old_out);
    return err;
  }
  void release() {  // at handle destruction
    if (stream) (void)hipStreamSynchronize(stream);
    for (char *p : {d_in, d_out, d_ws})
      if (p) (void)hipFree(p);
    for (char *p : {h_in, h_out})
      if (p) (void)hipHostFree(p);
    if (ev_start) (void)hipEventDestroy(ev_start);
    if (ev_done) (void)hipEventDestroy(ev_done);
    if (stream) (void)hipStreamDestroy(stream);
  }
};

// The GPU feeder's streams, events and buffers, kept on the handle between
// calls (pinned-memory and stream creation cost milliseconds per call).
struct Feeder {
  Slot slots[2];
  float *d_orient = nullptr;
  size_t orient_cap = 0;
  hipError_t init() {
    hipError_t e = hipSuccess;
    for (Slot &s : slots) {
      s.busy = false;  // nothing of an earlier (failed) call is scattered
      if (s.stream) {
        if (e == hipSuccess) e = hipStreamSynchronize(s.stream);
        continue;
      }
      if (e == hipSuccess) e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreate(&s.ev_start);
      if (e == hipSuccess) e = hipEventCreate(&s.ev_done);
    }
    return e;
  }
  hipError_t orient_upload(const float *orient, int O) {
    const size_t bytes = sizeof(float) * 12 * (size_t)O;
    if (bytes > orient_cap) {
      if (d_orient) (void)hipFree(d_orient);
      d_orient = nullptr;
      orient_cap = 0;
      hipError_t e = hipMalloc((void **)&d_orient, bytes);
      if (e != hipSuccess) return e;
      orient_cap = bytes;
    }
    return hipMemcpy(d_orient, orient, bytes, hipMemcpyHostToDevice);
  }
  static void release(void *p) {
    Feeder *f = (Feeder *)p;
    for (Slot &s : f->slots) s.release();
    if (f->d_orient) (void)hipFree(f->d_orient);
    delete f;
  }
};

}  // namespace

extern "C" int dock_batch_hybrid(dock_pocket *p, const dock_ligands *ligs, const float *orient,
                                 int n_orient, int angle_steps, const dock_params *prm,
                                 dock_results *out, const dock_hybrid_opts *opt,
                                 dock_hybrid_stats *stats) {
  if (!p || !ligs || !orient || !out || !opt) return abi_fail(DOCK_E_INVAL, "NULL argument");
  if (ligs->n_ligands > 0 && (!out->best_score || !out->best_orient || !out->xyz_out))
    return abi_fail(DOCK_E_INVAL, "result array is NULL");
  if (ligs->total_rot > 0 && !out->angle_idx) return abi_fail(DOCK_E_INVAL, "angle_idx is NULL");
  int max_n = 0, max_r = 0;
  int rc = dock::abi_check_sync(ligs, orient, n_orient, angle_steps, prm, &max_n, &max_r);
  if (rc) return rc;
  if (prm->mode != DOCK_MODE_PLAIN) return abi_fail(DOCK_E_INVAL, "hybrid calls run the plain sweep");
  if (prm->n_align != 0) return abi_fail(DOCK_E_INVAL, "hybrid calls take no alignment set");
  if (opt->gpu_chunk < 0 || opt->cpu_chunk < 0) return abi_fail(DOCK_E_INVAL, "negative chunk size");
  int threads = opt->cpu_threads;
  if (threads < 0) {
    const unsigned hw = std::thread::hardware_concurrency();
    threads = hw > 1 ? (int)hw - 1 : 0;  // one CPU drives the GPU
  }
  if (threads > 1024) return abi_fail(DOCK_E_LIMIT, "cpu_threads %d above 1024", threads);
  if (!opt->use_gpu && threads == 0) return abi_fail(DOCK_E_INVAL, "no GPU and no host threads");
  if (threads > 0 && !dock_cpu::supported())
    return abi_fail(DOCK_E_STATE, "host threads need a CPU with AVX2 and FMA");

  const int64_t L = ligs->n_ligands;
  const int O = n_orient, S = angle_steps, passes = prm->passes;
  const bool all = out->all_scores && out->all_angle_idx;
  if ((out->all_scores != nullptr) != (out->all_angle_idx != nullptr))
    return abi_fail(DOCK_E_INVAL, "hybrid calls return all_scores and all_angle_idx together");
  if (stats) {
    stats->gpu_ligands = stats->cpu_ligands = 0;
    stats->gpu_chunks = 0;
    stats->cpu_threads = threads;
    stats->wall_ms = stats->gpu_busy_ms = stats->cpu_busy_ms = stats->feed_ms = stats->wait_ms = 0.0;
  }
  if (L == 0) return DOCK_OK;
  const auto t_start = Clock::now();

  Dispenser disp;
  disp.back = L;

  dock::abi_lock(p);
  struct Unlock {
    dock_pocket *p;
    ~Unlock() { dock::abi_unlock(p); }
  } unlock{p};
  int dev_prev = -1;
  (void)hipGetDevice(&dev_prev);
  const int dev = dock::abi_device(p);
  if (dev_prev != dev) (void)hipSetDevice(dev);
  struct Restore {
    int prev, dev;
    ~Restore() {
      if (prev >= 0 && prev != dev) (void)hipSetDevice(prev);
    }
  } restore{dev_prev, dev};

  // host side: grid copy, (cos, sin) table, workers
  std::vector<float> cs(2 * (size_t)S);
  for (int k = 0; k < S; ++k) {
    const double th = 6.283185307179586476925286766559 * (double)k / (double)S;
    cs[2 * k] = (float)std::cos(th);
    cs[2 * k + 1] = (float)std::sin(th);
  }
  dock_cpu::Grid hg{};
  if (threads > 0) {
    dock::HostGrid g{};
    if ((rc = dock::abi_host_grid(p, &g)) != DOCK_OK) return rc;
    hg = dock_cpu::Grid{g.v, g.nx, g.ny, g.nz, g.ox, g.oy, g.oz, g.inv_h};
  }
  const dock_cpu::Batch hb{ligs->atom_offset, ligs->xyz, ligs->rot_offset, ligs->rot_axis,
                           ligs->move_offset, ligs->move_atoms};
  const dock_cpu::Params hp{orient, O, S, passes, prm->r_bump * prm->r_bump, cs.data()};
  const dock_cpu::Out ho{out->best_score, out->best_orient, out->angle_idx, out->xyz_out,
                         all ? out->all_scores : nullptr, all ? out->all_angle_idx : nullptr,
                         out->status};
  int8_t *done_by = stats ? stats->done_by : nullptr;
  const int64_t cpu_chunk = opt->cpu_chunk > 0 ? opt->cpu_chunk : 1;
  std::atomic<int64_t> cpu_done{0};
  std::atomic<int64_t> cpu_ns{0};
  std::vector<std::thread> pool;
  try {
    for (int t = 0; t < threads; ++t)
      pool.emplace_back([&]() {
        dock_cpu::Worker w;
        int64_t b, e, mine = 0;
        const auto t0 = Clock::now();
        while (disp.take_back(cpu_chunk, &b, &e))
          for (int64_t l = b; l < e; ++l) {
            w.dock_ligand(hg, hb, hp, (int)l, ho);
            if (done_by) done_by[l] = 1;
            ++mine;
          }
        cpu_ns += std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now() - t0).count();
        cpu_done += mine;
      });
  } catch (const std::exception &) {
    // take every range so started threads stop, then report
    int64_t b, e;
    while (disp.take_front(L, &b, &e)) {
    }
    for (auto &t : pool) t.join();
    return abi_fail(DOCK_E_NOMEM, "could not start host threads");
  }

  // GPU feeder
  int gpu_rc = DOCK_OK;
  int64_t gpu_done = 0;
  int chunks = 0;
  double gpu_ms = 0.0, feed_ms = 0.0, wait_ms = 0.0;
  if (opt->use_gpu) {
    // guided range sizes: a quarter of what is left, within [gmax / 4, gmax]
    const int64_t gmax = opt->gpu_chunk > 0 ? opt->gpu_chunk : std::max<int64_t>(256, (L + 3) / 4);
    const int64_t gmin = std::max<int64_t>(1, gmax / 4);
    dock::HybridCache *hc = dock::abi_hybrid_cache(p);
    if (!hc->state) {
      Feeder *f = new (std::nothrow) Feeder;
      if (f) {
        hc->state = f;
        hc->release = &Feeder::release;
      }
    }
    Feeder *feeder = (Feeder *)hc->state;
    hipError_t e = feeder ? feeder->init() : hipErrorOutOfMemory;
    if (e == hipSuccess) e = feeder->orient_upload(orient, O);
    if (e != hipSuccess) gpu_rc = hip_err(e, "hybrid GPU set-up");
    Slot *slots = feeder ? feeder->slots : nullptr;
    float *d_orient = feeder ? feeder->d_orient : nullptr;
    dock_params gp = *prm;
    gp.flags &= ~(uint32_t)(DOCK_FLAG_GRAPH | DOCK_FLAG_TIME_SWEEP);
    gp.max_atoms = max_n;
    gp.max_rot = 0;
    gp.align_rot = nullptr;

    // results of a finished slot into the caller's arrays
    auto scatter = [&](Slot &s) -> int {
      const auto tw = Clock::now();
      hipError_t err = hipEventSynchronize(s.ev_done);
      const auto ts = Clock::now();
      wait_ms += std::chrono::duration<double, std::milli>(ts - tw).count();
      struct Acc {
        Clock::time_point t;
        double *ms;
        ~Acc() { *ms += std::chrono::duration<double, std::milli>(Clock::now() - t).count(); }
      } acc{ts, &feed_ms};
      if (err != hipSuccess) return hip_err(err, "hybrid chunk");
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, s.ev_start, s.ev_done) == hipSuccess) gpu_ms += ms;
      const ChunkLayout &c = s.lay;
      const char *h = s.h_out;
      const int64_t b = s.b, n = s.e - s.b;
      const int64_t a0 = ligs->atom_offset[b], r0 = ligs->rot_offset[b];
      std::memcpy(out->best_score + b, h + c.bs, 4 * (size_t)n);
      std::memcpy(out->best_orient + b, h + c.bo, 4 * (size_t)n);
      if (out->status) std::memcpy(out->status + b, h + c.st, 4 * (size_t)n);
      if (c.NR) std::memcpy(out->angle_idx + r0 * passes, h + c.ai, 2 * (size_t)c.NR * passes);
      std::memcpy(out->xyz_out + 3 * a0, h + c.xo, 12 * (size_t)c.NA);
      if (all) {
        std::memcpy(out->all_scores + b * O, h + c.as, 4 * (size_t)n * O);
        if (c.NR)
          std::memcpy(out->all_angle_idx + r0 * O * passes, h + c.aai,
                      2 * (size_t)c.NR * O * passes);
      }
      if (done_by) std::memset(done_by + b, 0, (size_t)n);
      gpu_done += s.e - s.b;
      s.busy = false;
      return DOCK_OK;
    };

    int cur = 0;
    int64_t b, en;
    auto range = [&](int64_t *bb, int64_t *ee) {
      int64_t want;
      {
        std::lock_guard<std::mutex> lk(disp.mu);
        want = std::min(gmax, std::max(gmin, (disp.back - disp.front) / 4));
      }
      return disp.take_front(want, bb, ee);
    };
    while (gpu_rc == DOCK_OK && range(&b, &en)) {
      Slot &s = slots[cur];
      if (s.busy && (gpu_rc = scatter(s)) != DOCK_OK) break;
      const int64_t a0 = ligs->atom_offset[b], a1 = ligs->atom_offset[en];
      const int64_t r0 = ligs->rot_offset[b], r1 = ligs->rot_offset[en];
      const int64_t m0 = r1 > r0 ? ligs->move_offset[r0] : 0, m1 = r1 > r0 ? ligs->move_offset[r1] : 0;
      s.lay.plan(en - b, a1 - a0, r1 - r0, m1 - m0, O, S, passes, all);
      s.b = b;
      s.e = en;
      if ((e = s.grow(s.lay)) != hipSuccess) {
        gpu_rc = hip_err(e, "hybrid chunk buffers");
        break;
      }
      // pack the slice: offsets rebased to the slice, the rest copied as is
      const auto tp = Clock::now();
      const ChunkLayout &c = s.lay;
      char *h = s.h_in;
      int32_t *ao = (int32_t *)(h + c.ao), *ro = (int32_t *)(h + c.ro), *mo = (int32_t *)(h + c.mo);
      for (int64_t k = 0; k <= c.L; ++k) {
        ao[k] = (int32_t)(ligs->atom_offset[b + k] - a0);
        ro[k] = (int32_t)(ligs->rot_offset[b + k] - r0);
      }
      std::memcpy(h + c.xyz, ligs->xyz + 3 * a0, 12 * (size_t)c.NA);
      if (c.NR) {
        std::memcpy(h + c.ax, ligs->rot_axis + 2 * r0, 8 * (size_t)c.NR);
        for (int64_t k = 0; k <= c.NR; ++k) mo[k] = (int32_t)(ligs->move_offset[r0 + k] - m0);
      } else {
        mo[0] = 0;
      }
      if (c.NM) std::memcpy(h + c.mv, ligs->move_atoms + m0, 2 * (size_t)c.NM);
      feed_ms += std::chrono::duration<double, std::milli>(Clock::now() - tp).count();
      dock_ligands dl{(int32_t)c.L, c.NA, c.NR, c.NM,
                      (const int32_t *)(s.d_in + c.ao), (const float *)(s.d_in + c.xyz),
                      (const int32_t *)(s.d_in + c.ro), c.NR ? (const int32_t *)(s.d_in + c.ax) : nullptr,
                      c.NR ? (const int32_t *)(s.d_in + c.mo) : nullptr,
                      c.NM ? (const int16_t *)(s.d_in + c.mv) : nullptr};
      dock_results dr{};
      dr.best_score = (float *)(s.d_out + c.bs);
      dr.best_orient = (int32_t *)(s.d_out + c.bo);
      dr.angle_idx = c.NR ? (int16_t *)(s.d_out + c.ai) : nullptr;
      dr.xyz_out = (float *)(s.d_out + c.xo);
      dr.all_scores = all ? (float *)(s.d_out + c.as) : nullptr;
      dr.all_angle_idx = all && c.NR ? (int16_t *)(s.d_out + c.aai) : nullptr;
      dr.status = (int32_t *)(s.d_out + c.st);
      e = hipEventRecord(s.ev_start, s.stream);
      if (e == hipSuccess) e = hipMemcpyAsync(s.d_in, s.h_in, c.in_bytes, hipMemcpyHostToDevice, s.stream);
      if (e != hipSuccess) {
        gpu_rc = hip_err(e, "hybrid upload");
        break;
      }
      if ((gpu_rc = dock::abi_enqueue_plain(p, &dl, d_orient, O, S, &gp, &dr, s.d_ws, s.cap_ws,
                                            s.stream)) != DOCK_OK)
        break;
      e = hipMemcpyAsync(s.h_out, s.d_out, c.out_bytes, hipMemcpyDeviceToHost, s.stream);
      if (e == hipSuccess) e = hipEventRecord(s.ev_done, s.stream);
      if (e != hipSuccess) {
        gpu_rc = hip_err(e, "hybrid download");
        break;
      }
      s.busy = true;
      ++chunks;
      cur ^= 1;
    }
    for (int k = 0; k < 2 && slots; ++k) {
      Slot &s = slots[(cur + k) & 1];
      if (s.busy) {
        const int r2 = scatter(s);
        if (gpu_rc == DOCK_OK) gpu_rc = r2;
      }
    }
    if (gpu_rc != DOCK_OK) {  // stop the host threads: nothing more to take
      int64_t bb, ee;
      while (disp.take_front(L, &bb, &ee)) {
      }
    }
    if (slots)  // leave both streams idle for the next call
      for (int k = 0; k < 2; ++k)
        if (slots[k].stream) (void)hipStreamSynchronize(slots[k].stream);
  }
  for (auto &t : pool) t.join();
  if (gpu_rc != DOCK_OK) return gpu_rc;
  if (gpu_done + cpu_done.load() != L)
    return abi_fail(DOCK_E_DEVICE, "hybrid call finished %lld of %lld ligands",
                    (long long)(gpu_done + cpu_done.load()), (long long)L);
  if (stats) {
    stats->gpu_ligands = gpu_done;
    stats->cpu_ligands = cpu_done.load();
    stats->gpu_chunks = chunks;
    stats->wall_ms = std::chrono::duration<double, std::milli>(Clock::now() - t_start).count();
    stats->gpu_busy_ms = gpu_ms;
    stats->cpu_busy_ms = (double)cpu_ns.load() / 1e6;
    stats->feed_ms = feed_ms;
    stats->wait_ms = wait_ms;
  }
  return DOCK_OK;
}
