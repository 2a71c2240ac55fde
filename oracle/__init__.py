"""FP64 CPU reference of the greedy rotamer sweep -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its binding) never loads it and shares no code with it.

``liboracle.so`` (``oracle.cpp``) holds the reference itself; this module is
argument marshalling.  See ``oracle.cpp`` for the readings of the paper it
implements (paper §3.1, §4.1, Listings 1-2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
DELTA = 1e-4  # ambiguity band in A (voxel faces and the bump radius)

FLAG_VALID, FLAG_VAMB, FLAG_SAMB = 1, 2, 4

_lib = None


def build(force: bool = False) -> str:
    src = os.path.join(_HERE, "oracle.cpp")
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(src):
        tmp = LIB_PATH + ".tmp"
        subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-pthread",
                        src, "-o", tmp], check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        lib = ctypes.CDLL(LIB_PATH)
        c = ctypes
        P = c.c_void_p
        lib.oracle_rotate.argtypes = [P, P, c.c_double, P, P]
        lib.oracle_voxel_value.restype = c.c_double
        lib.oracle_voxel_value.argtypes = [P, c.c_int, c.c_int, c.c_int, P, c.c_float, P]
        lib.oracle_voxel_interval.argtypes = [P, c.c_int, c.c_int, c.c_int, P, c.c_float, P,
                                              c.c_double, P, P, P]
        lib.oracle_trace_item.argtypes = (
            [P, c.c_int, c.c_int, c.c_int, P, c.c_float, c.c_int, P, c.c_int, P, P, P, P,
             c.c_int, c.c_double, c.c_int, P, c.c_double, P, P, P, P, P, P, P, P, P,
             P, c.c_int, c.c_int, P, P, P, P, P])
        lib.oracle_dock_batch.argtypes = (
            [P, c.c_int, c.c_int, c.c_int, P, c.c_float, c.c_int, P, P, P, P, P, P, P,
             c.c_int, c.c_int, c.c_double, c.c_int, P, P, P, P, P, c.c_int,
             P, c.c_int, P, P])
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def rotate(a, u, theta, x):
    """Rodrigues rotation of point x by theta about the unit axis u through a."""
    a, u, x = (_c(v, np.float64) for v in (a, u, x))
    y = np.empty(3, np.float64)
    _load().oracle_rotate(_p(a), _p(u), float(theta), _p(x), _p(y))
    return y


def voxel_value(pocket, p) -> float:
    g = _c(pocket.grid, np.float32)
    nz, ny, nx = g.shape
    return _load().oracle_voxel_value(_p(g), nx, ny, nz, _p(_c(pocket.origin, np.float32)),
                                      float(pocket.spacing), _p(_c(p, np.float64)))


def voxel_interval(pocket, p, delta: float = DELTA):
    """(lo, hi, ambiguous): the range of voxel values a lookup of p can take if
    p moves by less than delta on each axis, and whether p lies within delta
    of a voxel face."""
    g = _c(pocket.grid, np.float32)
    nz, ny, nx = g.shape
    lo, hi = np.zeros(1), np.zeros(1)
    am = np.zeros(1, np.int32)
    _load().oracle_voxel_interval(_p(g), nx, ny, nz, _p(_c(pocket.origin, np.float32)),
                                  float(pocket.spacing), _p(_c(p, np.float64)), float(delta),
                                  _p(lo), _p(hi), _p(am))
    return float(lo[0]), float(hi[0]), bool(am[0])


@dataclass
class Trace:
    k_star: np.ndarray      # [steps] the reference's own argmax per step
    xyz: np.ndarray         # [n, 3] final pose along the followed trajectory
    score: float
    score_lo: float
    score_hi: float
    prof_s: np.ndarray      # [steps, S]
    prof_lo: np.ndarray
    prof_hi: np.ndarray
    prof_flags: np.ndarray  # uint8 bits: 1 valid, 2 validity ambiguous, 4 score ambiguous
    # rigid alignment (empty without a rotation set)
    a_star: int = -1            # the reference's own best rotation
    align_s: np.ndarray = None  # [n_align] score of every candidate rotation
    align_lo: np.ndarray = None
    align_hi: np.ndarray = None
    align_flags: np.ndarray = None  # uint8 bit 4: score ambiguous


def _rotations(align):
    if align is None:
        return None, 0
    a = _c(align, np.float32).reshape(-1, 9)
    return a, a.shape[0]


def trace_item(pocket, lig: dict, orient, S: int, r_bump: float = 2.0, passes: int = 1,
               forced_k=None, delta: float = DELTA, align=None, forced_a: int = -1) -> Trace:
    """One (ligand, orientation) restart with its full per-step record.

    align: optional [A, 3, 3] rotation set; the restart is first aligned
    rigidly (paper §3.1, §4.1) to the best of them about its centroid, or to
    rotation forced_a if that is >= 0."""
    g = _c(pocket.grid, np.float32)
    nz, ny, nx = g.shape
    xyz = _c(lig["xyz"], np.float32)
    n = xyz.shape[0]
    axis = _c(lig["rot_axis"], np.int32)
    R = axis.shape[0]
    moff = _c(lig["move_offset"], np.int32)
    mv = _c(lig["move_atoms"], np.int16)
    steps = R * passes
    k = np.empty(max(steps, 1), np.int16)
    xo = np.empty((n, 3), np.float64)
    fs, flo, fhi = (np.zeros(1, np.float64) for _ in range(3))
    ps, plo, phi = (np.empty((max(steps, 1), S), np.float64) for _ in range(3))
    pf = np.empty((max(steps, 1), S), np.uint8)
    fk = None if forced_k is None else _c(forced_k, np.int16)
    rot, A = _rotations(align)
    ast = np.full(1, -1, np.int16)
    als, alo, ahi = (np.empty(max(A, 1), np.float64) for _ in range(3))
    af = np.empty(max(A, 1), np.uint8)
    rc = _load().oracle_trace_item(
        _p(g), nx, ny, nz, _p(_c(pocket.origin, np.float32)), float(pocket.spacing), n,
        _p(xyz), R, _p(axis), _p(moff), _p(mv), _p(_c(orient, np.float32)), S,
        float(r_bump), passes, _p(fk), float(delta), _p(k), _p(xo), _p(fs), _p(flo),
        _p(fhi), _p(ps), _p(plo), _p(phi), _p(pf), _p(rot), A, int(forced_a), _p(ast),
        _p(als), _p(alo), _p(ahi), _p(af))
    if rc != 0:
        raise ValueError("oracle_trace_item: bad arguments")
    return Trace(k[:steps], xo, float(fs[0]), float(flo[0]), float(fhi[0]),
                 ps[:steps], plo[:steps], phi[:steps], pf[:steps], int(ast[0]),
                 als[:A], alo[:A], ahi[:A], af[:A])


@dataclass
class BatchResult:
    best_score: np.ndarray   # [L] f64
    best_orient: np.ndarray  # [L] i32
    angle_idx: np.ndarray    # [total_rot * passes] i16
    xyz: np.ndarray          # [total_atoms, 3] f64
    all_scores: np.ndarray   # [L, O] f64
    best_align: np.ndarray = None  # [L] i16, alignment of the best orientation (-1: none)
    all_align: np.ndarray = None   # [L, O] i16


def dock_batch(pocket, ligs, orient, S: int, r_bump: float = 2.0, passes: int = 1,
               n_threads: int = 0, align=None) -> BatchResult:
    """Every ligand x orientation restart; align: optional [A, 3, 3] rotation set."""
    g = _c(pocket.grid, np.float32)
    nz, ny, nx = g.shape
    orient = _c(orient, np.float32).reshape(-1, 12)
    L, O = ligs.n_ligands, orient.shape[0]
    rot, A = _rotations(align)
    out = BatchResult(np.empty(L), np.empty(L, np.int32),
                      np.empty(max(1, int(ligs.rot_offset[-1]) * passes), np.int16),
                      np.empty((ligs.xyz.shape[0], 3)), np.empty((L, O)),
                      np.full(max(L, 1), -1, np.int16), np.full((max(L, 1), O), -1, np.int16))
    rc = _load().oracle_dock_batch(
        _p(g), nx, ny, nz, _p(_c(pocket.origin, np.float32)), float(pocket.spacing), L,
        _p(_c(ligs.atom_offset, np.int32)), _p(_c(ligs.xyz, np.float32)),
        _p(_c(ligs.rot_offset, np.int32)), _p(_c(ligs.rot_axis, np.int32)),
        _p(_c(ligs.move_offset, np.int32)), _p(_c(ligs.move_atoms, np.int16)),
        _p(orient), O, S, float(r_bump), passes, _p(out.best_score), _p(out.best_orient),
        _p(out.angle_idx), _p(out.xyz), _p(out.all_scores), n_threads, _p(rot), A,
        _p(out.best_align), _p(out.all_align))
    if rc != 0:
        raise ValueError("oracle_dock_batch: bad arguments")
    out.angle_idx = out.angle_idx[:int(ligs.rot_offset[-1]) * passes]
    out.best_align, out.all_align = out.best_align[:L], out.all_align[:L]
    return out
