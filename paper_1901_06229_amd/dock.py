"""Python binding of libdock.so (include/dock.h): argument marshalling only.

Every step of the sweep runs in the HIP library.  There is no CPU fallback:
if ``libdock.so`` is missing or cannot be loaded, every call raises.
torch is used only for device memory and streams (``dock_batch_async``).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .build import LIB_PATH

DOCK_OK, DOCK_E_INVAL, DOCK_E_LIMIT, DOCK_E_NOMEM, DOCK_E_DEVICE, DOCK_E_CANCELLED, DOCK_E_STATE = \
    0, -1, -2, -3, -4, -5, -6
DOCK_MODE_PLAIN, DOCK_MODE_LEARNED = 0, 1
DOCK_FLAG_NO_LPT = 1
DOCK_FLAG_TIME_SWEEP = 2
DOCK_FLAG_DIRECT_BUMP = 4
DOCK_FLAG_GRAPH = 8
DOCK_MAX_ATOMS, DOCK_MAX_ROT, DOCK_MAX_STEPS = 256, 255, 4096
DOCK_STATIC_SCRATCH_BYTES = 64 << 20
DOCK_GROUP_MAX_STEPS = 2048

_P = ctypes.c_void_p


class dock_ligands(ctypes.Structure):
    _fields_ = [("n_ligands", ctypes.c_int32), ("total_atoms", ctypes.c_int64),
                ("total_rot", ctypes.c_int64), ("total_move", ctypes.c_int64),
                ("atom_offset", _P), ("xyz", _P), ("rot_offset", _P), ("rot_axis", _P),
                ("move_offset", _P), ("move_atoms", _P)]


class dock_params(ctypes.Structure):
    _fields_ = [("r_bump", ctypes.c_float), ("passes", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("top_k", ctypes.c_int32), ("margin", ctypes.c_float), ("flags", ctypes.c_uint32),
                ("max_atoms", ctypes.c_int32), ("max_rot", ctypes.c_int32),
                ("n_align", ctypes.c_int32), ("align_rot", _P)]


class dock_results(ctypes.Structure):
    _fields_ = [("best_score", _P), ("best_orient", _P), ("angle_idx", _P), ("xyz_out", _P),
                ("all_scores", _P), ("all_angle_idx", _P), ("status", _P), ("n_fallback", _P),
                ("align_idx", _P), ("all_align_idx", _P)]


class dock_tune_entry(ctypes.Structure):
    _fields_ = [("waves_per_block", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("items_per_claim", ctypes.c_int32), ("sweep_ms", ctypes.c_float),
                ("group16_atoms", ctypes.c_int32), ("group32_atoms", ctypes.c_int32),
                ("group32_split", ctypes.c_int32)]


class dock_hybrid_opts(ctypes.Structure):
    _fields_ = [("cpu_threads", ctypes.c_int32), ("use_gpu", ctypes.c_int32),
                ("gpu_chunk", ctypes.c_int32), ("cpu_chunk", ctypes.c_int32)]


class dock_hybrid_stats(ctypes.Structure):
    _fields_ = [("gpu_ligands", ctypes.c_int64), ("cpu_ligands", ctypes.c_int64),
                ("gpu_chunks", ctypes.c_int32), ("cpu_threads", ctypes.c_int32),
                ("wall_ms", ctypes.c_double), ("gpu_busy_ms", ctypes.c_double),
                ("cpu_busy_ms", ctypes.c_double), ("feed_ms", ctypes.c_double),
                ("wait_ms", ctypes.c_double), ("done_by", ctypes.c_void_p)]


class DockError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__(f"{where}: {detail or 'error'} (code {code})")
        self.code = code


_lib = None


def _bind_torch_runtime():
    """Load torch's HIP runtime first when torch is installed.

    torch ships its own libamdhip64 / libhsa-runtime64 (same sonames as the
    system ROCm).  Loading torch first makes libdock.so bind to that runtime,
    so one HIP runtime serves the whole process and torch's device memory and
    streams are valid handles for the library.  Without torch, libdock.so
    uses the system ROCm runtime.
    """
    try:
        import torch  # noqa: F401
    except ImportError:
        pass


def load_library(path: str = None):
    """Load libdock.so; raises if it is not built (no fallback path exists).

    PAPER_1901_06229_AMD_LIB may name another build of the same library.
    """
    global _lib
    if _lib is not None:
        return _lib
    path = path or os.environ.get("PAPER_1901_06229_AMD_LIB") or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run __graft_entry__.build() first")
    _bind_torch_runtime()
    lib = ctypes.CDLL(path)
    c = ctypes
    lib.dock_init_pocket.argtypes = [_P, c.c_int, c.c_int, c.c_int, _P, c.c_float, c.POINTER(_P)]
    lib.dock_init_pocket.restype = c.c_int
    lib.dock_free_pocket.argtypes = [_P]
    lib.dock_free_pocket.restype = None
    lib.dock_batch.argtypes = [_P, c.POINTER(dock_ligands), _P, c.c_int, c.c_int,
                               c.POINTER(dock_params), c.POINTER(dock_results)]
    lib.dock_batch.restype = c.c_int
    lib.dock_batch_async.argtypes = [_P, c.POINTER(dock_ligands), _P, c.c_int, c.c_int,
                                     c.POINTER(dock_params), c.POINTER(dock_results), _P,
                                     c.c_size_t, _P]
    lib.dock_batch_async.restype = c.c_int
    lib.dock_batch_async_static.argtypes = [_P, c.POINTER(dock_ligands), _P, c.c_int, c.c_int,
                                            c.POINTER(dock_params), c.POINTER(dock_results), _P]
    lib.dock_batch_async_static.restype = c.c_int
    lib.dock_batch_hybrid.argtypes = [_P, c.POINTER(dock_ligands), _P, c.c_int, c.c_int,
                                      c.POINTER(dock_params), c.POINTER(dock_results),
                                      c.POINTER(dock_hybrid_opts), c.POINTER(dock_hybrid_stats)]
    lib.dock_batch_hybrid.restype = c.c_int
    lib.dock_workspace_size.argtypes = [c.c_int32, c.c_int64, c.c_int, c.c_int, c.c_int, c.c_int]
    lib.dock_workspace_size.restype = c.c_size_t
    lib.dock_last_sweep_ms.argtypes = [_P, c.POINTER(c.c_float)]
    lib.dock_last_align_ms.restype = c.c_int
    lib.dock_last_align_ms.argtypes = [_P, c.POINTER(c.c_float)]
    lib.dock_probe_gather.restype = c.c_int
    lib.dock_probe_gather.argtypes = [_P, c.c_int, c.c_int, c.c_int, _P, c.POINTER(c.c_float), _P]
    lib.dock_last_sweep_ms.restype = c.c_int
    lib.dock_probe_valu.restype = c.c_int
    lib.dock_probe_valu.argtypes = [c.c_int, c.c_int, c.c_int, _P, c.POINTER(c.c_float), _P]
    lib.dock_sweep_ms_history.argtypes = [_P, c.c_int, c.POINTER(c.c_float)]
    lib.dock_sweep_ms_history.restype = c.c_int
    lib.dock_last_sweep_work.argtypes = [_P, c.POINTER(c.c_uint64), c.POINTER(c.c_uint64)]
    lib.dock_last_sweep_work.restype = c.c_int
    lib.dock_set_launch.argtypes = [_P, c.c_int, c.c_int, c.c_int]
    lib.dock_set_launch.restype = c.c_int
    lib.dock_get_launch.argtypes = [_P, c.POINTER(c.c_int), c.POINTER(c.c_int), c.POINTER(c.c_int)]
    lib.dock_get_launch.restype = c.c_int
    for name in ("dock_set_group_mapping",):
        getattr(lib, name).argtypes = [_P, c.c_int, c.c_int]
        getattr(lib, name).restype = c.c_int
    lib.dock_get_group_mapping.argtypes = [_P, c.POINTER(c.c_int), c.POINTER(c.c_int)]
    lib.dock_get_group_mapping.restype = c.c_int
    lib.dock_set_group_split.argtypes = [_P, c.c_int]
    lib.dock_set_group_split.restype = c.c_int
    lib.dock_get_group_split.argtypes = [_P, c.POINTER(c.c_int)]
    lib.dock_get_group_split.restype = c.c_int
    lib.dock_autotune.argtypes = [_P, c.POINTER(dock_ligands), _P, c.c_int, c.c_int,
                                  c.POINTER(dock_params), c.c_int, c.c_uint64,
                                  c.POINTER(dock_tune_entry), c.c_int, c.POINTER(c.c_int)]
    lib.dock_autotune.restype = c.c_int
    lib.dock_mlp_param_count.argtypes = []
    lib.dock_mlp_param_count.restype = c.c_size_t
    lib.dock_mlp_create.argtypes = [_P, c.POINTER(_P)]
    lib.dock_mlp_create.restype = c.c_int
    lib.dock_mlp_free.argtypes = [_P]
    lib.dock_mlp_free.restype = None
    for name in ("dock_mlp_get_params", "dock_mlp_set_params"):
        getattr(lib, name).argtypes = [_P, _P]
        getattr(lib, name).restype = c.c_int
    lib.dock_mlp_forward.argtypes = [_P, _P, c.c_int, _P, _P]
    lib.dock_mlp_forward.restype = c.c_int
    lib.dock_mlp_loss_grad.argtypes = [_P, _P, _P, c.c_int, _P, c.POINTER(c.c_float), _P]
    lib.dock_mlp_loss_grad.restype = c.c_int
    lib.dock_mlp_adam.argtypes = [_P, c.c_float, c.c_float, c.c_float, c.c_float, _P]
    lib.dock_mlp_adam.restype = c.c_int
    lib.dock_load_proposal.argtypes = [_P, _P]
    lib.dock_load_proposal.restype = c.c_int
    lib.dock_emit_profiles.argtypes = [_P, c.POINTER(dock_ligands), _P, c.c_int,
                                       c.POINTER(dock_params), _P, _P, _P]
    lib.dock_emit_profiles.restype = c.c_int
    lib.dock_strerror.argtypes = [c.c_int]
    lib.dock_strerror.restype = c.c_char_p
    lib.dock_last_error.argtypes = []
    lib.dock_last_error.restype = c.c_char_p
    _lib = lib
    return lib


def _check(rc: int, where: str):
    if rc != DOCK_OK:
        lib = load_library()
        raise DockError(rc, where, (lib.dock_last_error() or b"").decode() or
                        lib.dock_strerror(rc).decode())


def _np_ptr(a):
    return None if a is None else a.ctypes.data_as(_P)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


class Pocket:
    """Owns a dock_pocket handle (device copy of the grid)."""

    def __init__(self, handle, dims, origin, spacing):
        self.handle = handle
        self.dims = dims
        self.origin = origin
        self.spacing = spacing

    def close(self):
        if self.handle:
            load_library().dock_free_pocket(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dock_init_pocket(grid: np.ndarray, origin, spacing: float) -> Pocket:
    """grid: [nz, ny, nx] float32 (x fastest)."""
    lib = load_library()
    g = _c(grid, np.float32)
    nz, ny, nx = g.shape
    o = _c(origin, np.float32)
    h = _P()
    _check(lib.dock_init_pocket(_np_ptr(g), nx, ny, nz, _np_ptr(o), float(spacing),
                                ctypes.byref(h)), "dock_init_pocket")
    return Pocket(h, (nx, ny, nz), o.copy(), float(spacing))


def dock_free_pocket(p: Pocket):
    p.close()


def _any_ptr(a):
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return ctypes.c_void_p(a.data_ptr())
    return _np_ptr(a)


def make_params(r_bump=2.0, passes=1, mode=DOCK_MODE_PLAIN, top_k=16, margin=0.0, flags=0,
                max_atoms=0, max_rot=0, align=None) -> dock_params:
    """align: optional [A, 3, 3] float32 rotation set (a contiguous numpy array for
    dock_batch, a device tensor for dock_batch_async); the caller keeps it alive."""
    n_align = 0 if align is None else int(align.shape[0])
    return dock_params(float(r_bump), int(passes), int(mode), int(top_k), float(margin),
                       int(flags), int(max_atoms), int(max_rot), n_align, _any_ptr(align))


def _sync_call(ligs, orient, passes, mode, want_all, align, hybrid=False):
    """Host arrays of a synchronous call: (dock_ligands, dock_results, outputs,
    orientation table, arrays to keep alive)."""
    ao = _c(ligs.atom_offset, np.int32)
    xyz = _c(ligs.xyz, np.float32)
    ro = _c(ligs.rot_offset, np.int32)
    ax = _c(ligs.rot_axis, np.int32)
    mo = _c(ligs.move_offset, np.int32)
    mv = _c(ligs.move_atoms, np.int16)
    orient = _c(orient, np.float32).reshape(-1, 12)
    L, O = len(ao) - 1, orient.shape[0]
    NA, NR = int(ao[-1]) if L else 0, int(ro[-1]) if L else 0
    NM = int(mo[NR]) if NR else 0
    dl = dock_ligands(L, NA, NR, NM, _np_ptr(ao), _np_ptr(xyz), _np_ptr(ro), _np_ptr(ax),
                      _np_ptr(mo), _np_ptr(mv))
    out = dict(best_score=np.empty(L, np.float32), best_orient=np.empty(L, np.int32),
               angle_idx=np.empty(max(NR * passes, 1), np.int16),
               xyz=np.empty((max(NA, 1), 3), np.float32), status=np.empty(max(L, 1), np.int32))
    if want_all:
        out["all_scores"] = np.empty((L, O), np.float32)
        out["all_angle_idx"] = np.empty(max(NR * passes * O, 1), np.int16)
    if mode == DOCK_MODE_LEARNED and not hybrid:
        out["n_fallback"] = np.empty(max(L, 1), np.int32)
    if align is not None:
        align = _c(align, np.float32).reshape(-1, 3, 3)
        out["align_idx"] = np.empty(max(L, 1), np.int16)
        if want_all:
            out["all_align_idx"] = np.empty((max(L, 1), O), np.int16)
    dr = dock_results(_np_ptr(out["best_score"]), _np_ptr(out["best_orient"]),
                      _np_ptr(out["angle_idx"]), _np_ptr(out["xyz"]),
                      _np_ptr(out.get("all_scores")), _np_ptr(out.get("all_angle_idx")),
                      _np_ptr(out["status"]), _np_ptr(out.get("n_fallback")),
                      _np_ptr(out.get("align_idx")), _np_ptr(out.get("all_align_idx")))
    return dl, dr, out, orient, align, (ao, xyz, ro, ax, mo, mv), (L, O, NA, NR)


def _trim(out, sizes, passes, want_all, align):
    L, O, NA, NR = sizes
    out["angle_idx"] = out["angle_idx"][:NR * passes]
    out["xyz"] = out["xyz"][:NA]
    out["status"] = out["status"][:L]
    if want_all:
        out["all_angle_idx"] = out["all_angle_idx"][:NR * passes * O]
    if align is not None:
        out["align_idx"] = out["align_idx"][:L]
        if want_all:
            out["all_align_idx"] = out["all_align_idx"][:L]
    return out


def dock_batch(pocket: Pocket, ligs, orient, angle_steps: int, r_bump: float = 2.0,
               passes: int = 1, mode: int = DOCK_MODE_PLAIN, top_k: int = 16,
               margin: float = 0.0, flags: int = 0, want_all: bool = False, align=None) -> dict:
    """Synchronous batch on host arrays (``ligs``: any object with the CSR fields).

    align: optional [A, 3, 3] rotation set; every restart is first aligned
    rigidly to its best rotation (``align_idx`` per ligand, ``all_align_idx``
    per item with want_all)."""
    lib = load_library()
    dl, dr, out, orient, align, _keep, sizes = _sync_call(ligs, orient, passes, mode, want_all, align)
    prm = make_params(r_bump, passes, mode, top_k, margin, flags, align=align)
    _check(lib.dock_batch(pocket.handle, ctypes.byref(dl), _np_ptr(orient), sizes[1],
                          int(angle_steps), ctypes.byref(prm), ctypes.byref(dr)), "dock_batch")
    return _trim(out, sizes, passes, want_all, align)


def dock_batch_hybrid(pocket: Pocket, ligs, orient, angle_steps: int, r_bump: float = 2.0,
                      passes: int = 1, cpu_threads: int = -1, use_gpu: bool = True,
                      gpu_chunk: int = 0, cpu_chunk: int = 0, want_all: bool = False,
                      mode: int = DOCK_MODE_PLAIN, align=None) -> dict:
    """Synchronous batch docked by the GPU and host threads from one dispenser.
    Returns the dock_batch outputs plus ``stats`` (a dict) and ``done_by``
    (per ligand: 0 GPU, 1 host thread)."""
    lib = load_library()
    dl, dr, out, orient, align, _keep, sizes = _sync_call(ligs, orient, passes, mode, want_all, align,
                                                          hybrid=True)
    prm = make_params(r_bump, passes, mode, align=align)
    done_by = np.full(max(sizes[0], 1), -1, np.int8)
    opts = dock_hybrid_opts(int(cpu_threads), int(bool(use_gpu)), int(gpu_chunk), int(cpu_chunk))
    st = dock_hybrid_stats()
    st.done_by = done_by.ctypes.data
    _check(lib.dock_batch_hybrid(pocket.handle, ctypes.byref(dl), _np_ptr(orient), sizes[1],
                                 int(angle_steps), ctypes.byref(prm), ctypes.byref(dr),
                                 ctypes.byref(opts), ctypes.byref(st)), "dock_batch_hybrid")
    out = _trim(out, sizes, passes, want_all, align)
    out["done_by"] = done_by[:sizes[0]]
    out["stats"] = {k: getattr(st, k) for k, _ in dock_hybrid_stats._fields_ if k != "done_by"}
    return out


def dock_workspace_size(n_ligands: int, total_rot: int, n_orient: int, angle_steps: int,
                        passes: int = 1, n_align: int = 0) -> int:
    return int(load_library().dock_workspace_size(n_ligands, total_rot, n_orient, angle_steps,
                                                  passes, n_align))


def dock_last_sweep_ms(pocket: Pocket) -> float:
    ms = ctypes.c_float()
    _check(load_library().dock_last_sweep_ms(pocket.handle, ctypes.byref(ms)), "dock_last_sweep_ms")
    return float(ms.value)


def dock_sweep_ms_history(pocket: Pocket, n: int) -> list[float]:
    """Sweep durations (ms) of the last n timed calls on the handle, oldest first."""
    ms = (ctypes.c_float * max(int(n), 1))()
    _check(load_library().dock_sweep_ms_history(pocket.handle, int(n), ms), "dock_sweep_ms_history")
    return [float(x) for x in ms[:n]]


def dock_last_align_ms(pocket: Pocket) -> float:
    ms = ctypes.c_float()
    _check(load_library().dock_last_align_ms(pocket.handle, ctypes.byref(ms)), "dock_last_align_ms")
    return float(ms.value)


def dock_probe_gather(buf, out, log2_floats: int, blocks: int, iters: int, stream=None) -> float:
    """Random 4-byte gathers from buf (device tensor of >= 2^log2_floats floats) by
    blocks x 256 threads, iters each; out: device tensor of blocks * 256 floats.
    Returns the kernel's duration in ms."""
    ms = ctypes.c_float()
    st = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
    _check(load_library().dock_probe_gather(_tptr(buf), int(log2_floats), int(blocks), int(iters),
                                            _tptr(out), ctypes.byref(ms), st), "dock_probe_gather")
    return float(ms.value)


def dock_probe_valu(out, kind: int, blocks: int, iters: int, stream=None) -> float:
    """VALU issue probe (kind 0: FP32 FMA chains; 1: the sweep's evaluation
    mix); out: device tensor of blocks * 256 floats.  Returns the kernel's ms."""
    ms = ctypes.c_float()
    st = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
    _check(load_library().dock_probe_valu(int(kind), int(blocks), int(iters), _tptr(out),
                                          ctypes.byref(ms), st), "dock_probe_valu")
    return float(ms.value)


def dock_last_sweep_work(pocket: Pocket) -> tuple[int, int]:
    """(kept cross pairs, (moving atom, angle) evaluations) of the last timed sweep."""
    kp, ev = ctypes.c_uint64(), ctypes.c_uint64()
    _check(load_library().dock_last_sweep_work(pocket.handle, ctypes.byref(kp), ctypes.byref(ev)),
           "dock_last_sweep_work")
    return int(kp.value), int(ev.value)


def dock_set_launch(pocket: Pocket, waves_per_block: int = 0, blocks_per_cu: int = 0,
                    items_per_claim: int = 16):
    _check(load_library().dock_set_launch(pocket.handle, int(waves_per_block), int(blocks_per_cu),
                                          int(items_per_claim)), "dock_set_launch")


def dock_get_launch(pocket: Pocket):
    w, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(load_library().dock_get_launch(pocket.handle, ctypes.byref(w), ctypes.byref(b),
                                          ctypes.byref(c)), "dock_get_launch")
    return int(w.value), int(b.value), int(c.value)


def _host_ligands(ligs):
    keep = dict(ao=_c(ligs.atom_offset, np.int32), xyz=_c(ligs.xyz, np.float32),
                ro=_c(ligs.rot_offset, np.int32), ax=_c(ligs.rot_axis, np.int32),
                mo=_c(ligs.move_offset, np.int32), mv=_c(ligs.move_atoms, np.int16))
    L = len(keep["ao"]) - 1
    NA, NR = (int(keep["ao"][-1]), int(keep["ro"][-1])) if L else (0, 0)
    NM = int(keep["mo"][NR]) if NR else 0
    dl = dock_ligands(L, NA, NR, NM, _np_ptr(keep["ao"]), _np_ptr(keep["xyz"]),
                      _np_ptr(keep["ro"]), _np_ptr(keep["ax"]), _np_ptr(keep["mo"]),
                      _np_ptr(keep["mv"]))
    return dl, keep


def dock_autotune(pocket: Pocket, ligs, orient, angle_steps: int, sample_ligands: int,
                  seed: int = 0, **param_kw):
    """Time every candidate mapping on a seeded subset; keeps the fastest on the handle."""
    lib = load_library()
    dl, keep = _host_ligands(ligs)
    orient = _c(orient, np.float32).reshape(-1, 12)
    prm = make_params(**param_kw)
    entries = (dock_tune_entry * 256)()
    n = ctypes.c_int()
    _check(lib.dock_autotune(pocket.handle, ctypes.byref(dl), _np_ptr(orient), orient.shape[0],
                             int(angle_steps), ctypes.byref(prm), int(sample_ligands), int(seed),
                             entries, 256, ctypes.byref(n)), "dock_autotune")
    return [dict(waves_per_block=e.waves_per_block, blocks_per_cu=e.blocks_per_cu,
                 items_per_claim=e.items_per_claim, sweep_ms=e.sweep_ms,
                 group16_atoms=e.group16_atoms, group32_atoms=e.group32_atoms,
                 group32_split=e.group32_split)
            for e in entries[:n.value]]


def dock_set_group_mapping(pocket: Pocket, atoms16: int = 0, atoms32: int = 0):
    """Size classes docked 4 (<= atoms16 atoms) and 2 (<= atoms32) orientations
    per wave; 0 disables a class."""
    _check(load_library().dock_set_group_mapping(pocket.handle, int(atoms16), int(atoms32)),
           "dock_set_group_mapping")


def dock_get_group_mapping(pocket: Pocket):
    a, b = ctypes.c_int(), ctypes.c_int()
    _check(load_library().dock_get_group_mapping(pocket.handle, ctypes.byref(a), ctypes.byref(b)),
           "dock_get_group_mapping")
    return int(a.value), int(b.value)


def dock_set_group_split(pocket: Pocket, atoms: int = 0):
    """32-lane ligands in classes `atoms` wide, a kernel each (0: one class)."""
    _check(load_library().dock_set_group_split(pocket.handle, int(atoms)), "dock_set_group_split")


def dock_get_group_split(pocket: Pocket):
    a = ctypes.c_int()
    _check(load_library().dock_get_group_split(pocket.handle, ctypes.byref(a)),
           "dock_get_group_split")
    return int(a.value)


def _tptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _async_structs(dev: dict, out: dict):
    dl = dock_ligands(int(dev["n_ligands"]), int(dev["total_atoms"]), int(dev["total_rot"]),
                      int(dev["total_move"]), _tptr(dev["atom_offset"]), _tptr(dev["xyz"]),
                      _tptr(dev["rot_offset"]), _tptr(dev.get("rot_axis")),
                      _tptr(dev.get("move_offset")), _tptr(dev.get("move_atoms")))
    dr = dock_results(_tptr(out["best_score"]), _tptr(out["best_orient"]),
                      _tptr(out.get("angle_idx")), _tptr(out["xyz"]),
                      _tptr(out.get("all_scores")), _tptr(out.get("all_angle_idx")),
                      _tptr(out.get("status")), _tptr(out.get("n_fallback")),
                      _tptr(out.get("align_idx")), _tptr(out.get("all_align_idx")))
    return dl, dr


def dock_batch_async(pocket: Pocket, dev: dict, orient_dev, angle_steps: int, out: dict,
                     params: dock_params, workspace=None, stream=None):
    """Enqueue a batch whose arrays are device tensors (torch) on ``stream``.

    dev: atom_offset, xyz, rot_offset, rot_axis, move_offset, move_atoms (device
    tensors) and the python ints n_ligands, total_atoms, total_rot, total_move.
    out: best_score, best_orient, angle_idx, xyz (device tensors) and optional
    all_scores, all_angle_idx, status, n_fallback, align_idx, all_align_idx.
    """
    lib = load_library()
    dl, dr = _async_structs(dev, out)
    n_orient = int(orient_dev.shape[0])
    ws_ptr = _tptr(workspace)
    ws_bytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    st = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
    _check(lib.dock_batch_async(pocket.handle, ctypes.byref(dl), _tptr(orient_dev), n_orient,
                                int(angle_steps), ctypes.byref(params), ctypes.byref(dr), ws_ptr,
                                ws_bytes, st), "dock_batch_async")


def dock_batch_async_static(pocket: Pocket, dev: dict, orient_dev, angle_steps: int, out: dict,
                            params: dock_params, stream=None):
    """dock_batch_async in plain mode on the library's fixed per-device
    workspace: allocates nothing (batches needing more than
    DOCK_STATIC_SCRATCH_BYTES of workspace are refused)."""
    lib = load_library()
    dl, dr = _async_structs(dev, out)
    st = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
    _check(lib.dock_batch_async_static(pocket.handle, ctypes.byref(dl), _tptr(orient_dev),
                                       int(orient_dev.shape[0]), int(angle_steps),
                                       ctypes.byref(params), ctypes.byref(dr), st),
           "dock_batch_async_static")


# ---------------------------------------------------------------- learned proposal
class Mlp:
    """Owns a dock_mlp (the learned-proposal network on the current device)."""

    def __init__(self, params: np.ndarray):
        lib = load_library()
        p = _c(params, np.float32)
        if p.size != mlp_param_count():
            raise ValueError(f"expected {mlp_param_count()} parameters, got {p.size}")
        h = _P()
        _check(lib.dock_mlp_create(_np_ptr(p), ctypes.byref(h)), "dock_mlp_create")
        self.handle = h

    def close(self):
        if self.handle:
            load_library().dock_mlp_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self) -> np.ndarray:
        out = np.empty(mlp_param_count(), np.float32)
        _check(load_library().dock_mlp_get_params(self.handle, _np_ptr(out)), "dock_mlp_get_params")
        return out

    def set_params(self, params):
        p = _c(params, np.float32)
        _check(load_library().dock_mlp_set_params(self.handle, _np_ptr(p)), "dock_mlp_set_params")

    def forward(self, x_bf16, y_f32, stream=None):
        """x_bf16: device int16/bfloat16 tensor [rows, 64]; y_f32: device [rows, 256]."""
        st = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
        _check(load_library().dock_mlp_forward(self.handle, _tptr(x_bf16), int(x_bf16.shape[0]),
                                               _tptr(y_f32), st), "dock_mlp_forward")

    def loss_grad(self, x_bf16, t_bf16, grad_out=None, stream=None, want_loss=True):
        st = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
        loss = ctypes.c_float()
        _check(load_library().dock_mlp_loss_grad(
            self.handle, _tptr(x_bf16), _tptr(t_bf16), int(x_bf16.shape[0]), _tptr(grad_out),
            ctypes.byref(loss) if want_loss else None, st), "dock_mlp_loss_grad")
        return float(loss.value) if want_loss else None

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        st = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
        _check(load_library().dock_mlp_adam(self.handle, float(lr), float(beta1), float(beta2),
                                            float(eps), st), "dock_mlp_adam")


def mlp_param_count() -> int:
    return int(load_library().dock_mlp_param_count())


def dock_load_proposal(pocket: Pocket, mlp: Mlp):
    _check(load_library().dock_load_proposal(pocket.handle, mlp.handle), "dock_load_proposal")


def dock_emit_profiles(pocket: Pocket, ligs, orient, x_out, t_out, mask_out, r_bump=2.0,
                       passes=1):
    """Plain sweep (S = 256) writing per-step features, landscapes and masks
    into device tensors of total_rot*passes*n_orient rows."""
    lib = load_library()
    dl, keep = _host_ligands(ligs)
    orient = _c(orient, np.float32).reshape(-1, 12)
    prm = make_params(r_bump=r_bump, passes=passes)
    _check(lib.dock_emit_profiles(pocket.handle, ctypes.byref(dl), _np_ptr(orient), orient.shape[0],
                                  ctypes.byref(prm), _tptr(x_out), _tptr(t_out), _tptr(mask_out)),
           "dock_emit_profiles")
