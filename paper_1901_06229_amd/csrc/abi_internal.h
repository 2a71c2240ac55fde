// Hooks of the host runtime (dock_abi.hip) used by the other host-side
// translation units of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "dock.h"

namespace dock {

int abi_fail(int code, const char *fmt, ...);

// Host-side validation of a synchronous call's arguments (the checks of
// dock_batch): parameters, the CSR batch, finite coordinates and
// orientations.  max_n / max_r receive the largest atom and rotamer counts.
int abi_check_sync(const dock_ligands *ligs, const float *orient, int n_orient, int angle_steps,
                   const dock_params *prm, int *max_n, int *max_r);

// Enqueue one plain-mode batch (every pointer a device pointer) on st with
// a caller workspace; the caller holds the handle's lock.
int abi_enqueue_plain(dock_pocket *p, const dock_ligands *ligs, const float *orient, int n_orient,
                      int angle_steps, const dock_params *prm, const dock_results *out, void *ws,
                      size_t ws_bytes, hipStream_t st);

// The handle's device, and a host copy of its grid (copied back from the
// device on first use and cached on the handle; the caller holds the lock).
int abi_device(const dock_pocket *p);
struct HostGrid {
  const float *v;
  int nx, ny, nz;
  float ox, oy, oz, inv_h;
};
int abi_host_grid(dock_pocket *p, HostGrid *g);

// State the hybrid entry point keeps on a handle between calls (its streams
// and chunk buffers); freed with the handle through the stored deleter.
struct HybridCache {
  void *state = nullptr;
  void (*release)(void *) = nullptr;
};
HybridCache *abi_hybrid_cache(dock_pocket *p);

// The handle's lock (synchronous calls hold it for their whole duration).
void abi_lock(dock_pocket *p);
void abi_unlock(dock_pocket *p);

}  // namespace dock
