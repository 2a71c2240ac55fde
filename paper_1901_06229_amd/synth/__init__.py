"""Seeded synthetic inputs (pocket grids, ligand batches, orientations).

Thin ctypes wrapper over ``libdocksynth.so`` (built from ``synth.cpp``).  This
module is shared, as data, by the FP64 reference and the GPU path; it holds
none of the sweep's arithmetic.

Workload presets stand in for the paper's unpublished 1500-ligand library
(paper §5): the configurations below fix pocket size, ligand-size and
rotamer-count distributions, orientation count and angle steps.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdocksynth.so")

R_BUMP = 2.0  # bump radius in A, shared by every preset

# config id -> (n_ligands, n_orient, angle_steps, description)
PRESETS = {
    1: dict(n_ligands=1, n_orient=8, angle_steps=64,
            desc="64^3 pocket at 0.5 A, 1 ligand of 32 atoms, 4 rotamers"),
    2: dict(n_ligands=10_000, n_orient=256, angle_steps=256,
            desc="128^3 pocket at 0.375 A, 10k ligands (20-80 atoms, 2-12 rotamers)"),
    3: dict(n_ligands=100_000, n_orient=128, angle_steps=128,
            desc="128^3 pocket, 100k ligands (lognormal 8-150 atoms, 0-40 rotamers)"),
    4: dict(n_ligands=10_000, n_orient=8, angle_steps=256,
            desc="64^3 pocket, 32-atom 4-rotamer ligands; learned proposal"),
    5: dict(n_ligands=2_000, n_orient=64, angle_steps=360,
            desc="256^3 irregular pocket at 0.25 A, 2k ligands (100-250 atoms, 60-120 rotamers)"),
}

# generator streams
STREAM_POCKET, STREAM_LIGANDS, STREAM_ORIENT, STREAM_TRAIN, STREAM_EVAL = 0, 1, 2, 3, 4
STREAM_ALIGN = 5

_lib = None


def build(force: bool = False) -> str:
    """Compile libdocksynth.so with g++ (plain host code)."""
    import subprocess
    src = os.path.join(_HERE, "synth.cpp")
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
        lib.synth_ligands_create.restype = c.c_void_p
        lib.synth_ligands_create.argtypes = [c.c_int, c.c_uint64, c.c_int, c.c_int64,
                                             c.c_int64, c.c_double, c.c_int]
        lib.synth_ligands_sizes.argtypes = [c.c_void_p] + [c.POINTER(c.c_int64)] * 4
        lib.synth_ligands_copy.argtypes = [c.c_void_p] + [c.c_void_p] * 8
        lib.synth_ligands_free.argtypes = [c.c_void_p]
        lib.synth_pocket_shape.argtypes = [c.c_int, c.POINTER(c.c_int),
                                           c.POINTER(c.c_float), c.c_void_p]
        lib.synth_pocket_fill.argtypes = [c.c_int, c.c_uint64, c.c_void_p, c.c_int]
        lib.synth_orientations.argtypes = [c.c_uint64, c.c_int, c.c_int64, c.c_int64,
                                           c.c_void_p]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Pocket:
    grid: np.ndarray      # [G, G, G] float32, index [iz, iy, ix] (x fastest)
    origin: np.ndarray    # [3] float32, corner of voxel (0,0,0)
    spacing: float

    @property
    def dims(self):
        nz, ny, nx = self.grid.shape
        return nx, ny, nz


@dataclass
class Ligands:
    atom_offset: np.ndarray  # [L+1] int32
    xyz: np.ndarray          # [total_atoms, 3] float32
    rot_offset: np.ndarray   # [L+1] int32
    rot_axis: np.ndarray     # [total_rot, 2] int32, local (a, b); b on the moving side
    move_offset: np.ndarray  # [total_rot+1] int32
    move_atoms: np.ndarray   # [total_move] int16, local indices, ascending per rotamer
    eligible: np.ndarray     # [L] int32, eligible rotatable bonds per ligand
    r_target: np.ndarray     # [L] int32, rotamer count drawn before clipping

    @property
    def n_ligands(self) -> int:
        return len(self.atom_offset) - 1

    def n_atoms(self, l: int) -> int:
        return int(self.atom_offset[l + 1] - self.atom_offset[l])

    def n_rot(self, l: int) -> int:
        return int(self.rot_offset[l + 1] - self.rot_offset[l])

    def ligand(self, l: int) -> dict:
        """Arrays of one ligand, rebased to local offsets."""
        a0, a1 = self.atom_offset[l], self.atom_offset[l + 1]
        r0, r1 = self.rot_offset[l], self.rot_offset[l + 1]
        m0, m1 = self.move_offset[r0], self.move_offset[r1]
        return dict(xyz=self.xyz[a0:a1].copy(),
                    rot_axis=self.rot_axis[r0:r1].copy(),
                    move_offset=(self.move_offset[r0:r1 + 1] - m0).astype(np.int32),
                    move_atoms=self.move_atoms[m0:m1].copy())

    def subset(self, idx) -> "Ligands":
        """A new batch holding ligands idx (in that order)."""
        parts = [self.ligand(int(l)) for l in idx]
        return Ligands.from_parts(parts, self.eligible[list(idx)], self.r_target[list(idx)])

    @staticmethod
    def from_parts(parts, eligible=None, r_target=None) -> "Ligands":
        ao, ro, mo = [0], [0], [0]
        xyz, axis, mv = [], [], []
        for p in parts:
            ao.append(ao[-1] + len(p["xyz"]))
            xyz.append(np.asarray(p["xyz"], np.float32).reshape(-1, 3))
            R = len(p["rot_axis"])
            ro.append(ro[-1] + R)
            axis.append(np.asarray(p["rot_axis"], np.int32).reshape(-1, 2))
            moff = np.asarray(p["move_offset"], np.int64)
            for r in range(R):
                mo.append(mo[-1] + int(moff[r + 1] - moff[r]))
            mv.append(np.asarray(p["move_atoms"], np.int16))
        L = len(parts)
        return Ligands(
            atom_offset=np.asarray(ao, np.int32),
            xyz=np.concatenate(xyz) if xyz else np.zeros((0, 3), np.float32),
            rot_offset=np.asarray(ro, np.int32),
            rot_axis=np.concatenate(axis) if axis else np.zeros((0, 2), np.int32),
            move_offset=np.asarray(mo, np.int32),
            move_atoms=np.concatenate(mv) if mv else np.zeros(0, np.int16),
            eligible=np.zeros(L, np.int32) if eligible is None else np.asarray(eligible, np.int32),
            r_target=np.zeros(L, np.int32) if r_target is None else np.asarray(r_target, np.int32),
        )


def config_seed(config: int) -> int:
    return int(config)


def pocket(config: int, seed: int | None = None, n_threads: int = 0) -> Pocket:
    """Pocket grid of a config recipe (configs 1 and 4 share the 64^3 recipe)."""
    lib = _load()
    G = ctypes.c_int()
    h = ctypes.c_float()
    origin = np.zeros(3, np.float32)
    if lib.synth_pocket_shape(config, ctypes.byref(G), ctypes.byref(h), _ptr(origin)) != 0:
        raise ValueError(f"unknown pocket config {config}")
    grid = np.empty((G.value,) * 3, np.float32)
    s = config_seed(1 if config == 4 else config) if seed is None else seed
    lib.synth_pocket_fill(config, s, _ptr(grid), n_threads)
    return Pocket(grid=grid, origin=origin, spacing=float(h.value))


def ligands(config: int, count: int | None = None, first: int = 0, seed: int | None = None,
            stream: int = STREAM_LIGANDS, n_threads: int = 0) -> Ligands:
    lib = _load()
    if count is None:
        count = PRESETS[config]["n_ligands"]
    s = config_seed(config) if seed is None else seed
    h = lib.synth_ligands_create(config, s, stream, first, count, R_BUMP, n_threads)
    if not h:
        raise RuntimeError("ligand generation failed")
    try:
        sz = [ctypes.c_int64() for _ in range(4)]
        lib.synth_ligands_sizes(h, *[ctypes.byref(x) for x in sz])
        L, na, nr, nm = (x.value for x in sz)
        out = Ligands(atom_offset=np.empty(L + 1, np.int32), xyz=np.empty((na, 3), np.float32),
                      rot_offset=np.empty(L + 1, np.int32), rot_axis=np.empty((nr, 2), np.int32),
                      move_offset=np.empty(nr + 1, np.int32), move_atoms=np.empty(nm, np.int16),
                      eligible=np.empty(L, np.int32), r_target=np.empty(L, np.int32))
        lib.synth_ligands_copy(h, _ptr(out.atom_offset), _ptr(out.xyz), _ptr(out.rot_offset),
                               _ptr(out.rot_axis), _ptr(out.move_offset), _ptr(out.move_atoms),
                               _ptr(out.eligible), _ptr(out.r_target))
    finally:
        lib.synth_ligands_free(h)
    return out


def orientations(config: int, n: int | None = None, seed: int | None = None,
                 stream: int = STREAM_ORIENT, first: int = 0) -> np.ndarray:
    """[n, 12] float32 rigid transforms: row-major R then t (= 0)."""
    lib = _load()
    if n is None:
        n = PRESETS[config]["n_orient"]
    s = config_seed(config) if seed is None else seed
    out = np.empty((n, 12), np.float32)
    lib.synth_orientations(s, stream, first, n, _ptr(out))
    return out


def align_rotations(config: int, n: int, seed: int | None = None) -> np.ndarray:
    """[n, 3, 3] float32 rotation set for the rigid alignment search: the
    identity first (so an aligned restart never scores below its starting
    pose), then n - 1 uniform random rotations from their own stream."""
    out = np.empty((n, 3, 3), np.float32)
    if n > 0:
        out[0] = np.eye(3, dtype=np.float32)
    if n > 1:
        out[1:] = orientations(config, n - 1, seed=seed, stream=STREAM_ALIGN)[:, :9].reshape(-1, 3, 3)
    return out
