"""Hybrid host + GPU docking (dock_batch_hybrid) through the C-ABI.

The host threads' FP32 sweep is checked against the FP64 reference item by
item (the replay checker, the same bar as the GPU sweep); ligands the GPU
docks inside a hybrid call must equal the plain synchronous call bit for bit
(same kernels, results independent of the batch around them); every ligand
is docked exactly once.
"""
import numpy as np
import pytest

from paper_1901_06229_amd import dock, synth
from tests.checker import check_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pockets():
    cache = {}

    def get(cfg):
        if cfg not in cache:
            p = synth.pocket(cfg)
            cache[cfg] = (p, dock.dock_init_pocket(p.grid, p.origin, p.spacing))
        return cache[cfg]
    yield get
    for _, h in cache.values():
        h.close()


def _host_only(pockets, cfg, ligs, orient, S, passes=1, threads=4):
    p, h = pockets(cfg)
    print(f"[hybrid] host threads only, config {cfg}: {ligs.n_ligands} ligands x "
          f"{orient.shape[0]} orientations, S={S}, passes={passes}", flush=True)
    res = dock.dock_batch_hybrid(h, ligs, orient, S, passes=passes, cpu_threads=threads,
                                 use_gpu=False, want_all=True)
    assert (res["done_by"] == 1).all()
    assert res["stats"]["cpu_ligands"] == ligs.n_ligands and res["stats"]["gpu_ligands"] == 0
    assert (res["status"] == 0).all()
    rep = check_batch(p, ligs, orient, S, res, passes=passes)
    print(rep.summary())
    assert rep.ok(), rep.summary()
    rep.assert_rare()
    return res


def test_host_sweep_matches_reference_small(pockets):
    _host_only(pockets, 1, synth.ligands(1), synth.orientations(1), 64)
    _host_only(pockets, 1, synth.ligands(1), synth.orientations(1), 64, passes=3)


def test_host_sweep_matches_reference_batched(pockets):
    _host_only(pockets, 2, synth.ligands(2, count=24, first=500), synth.orientations(2, 12), 256)
    _host_only(pockets, 3, synth.ligands(3, count=60, first=900), synth.orientations(3, 8), 128)


def test_host_sweep_matches_reference_large_ligands(pockets):
    _host_only(pockets, 5, synth.ligands(5, count=3, first=40), synth.orientations(5, 2), 360)


def test_host_sweep_step_counts(pockets):
    """Angle-step counts around the 64-bit mask words and the 8-wide blocks."""
    ligs = synth.ligands(2, count=6, first=77)
    for S in (1, 7, 63, 64, 65, 129):
        _host_only(pockets, 2, ligs, synth.orientations(2, 4), S, threads=2)


def test_host_sweep_edge_cases(pockets):
    """No rotamers, one atom, an empty moving set."""
    from tests.helpers import make_lig
    import oracle
    p, h = pockets(1)
    one = make_lig(np.array([[0.5, 0.2, -0.3]], np.float32), [])
    xyz = np.array([[0, 0, 0], [1.5, 0, 0], [2.0, 1.4, 0], [3.5, 1.5, 0.3]], np.float32)
    rigid = make_lig(xyz, [])
    empty_move = make_lig(xyz, [(0, 1, [])])
    chain = make_lig(xyz, [(1, 2, [3])])
    ligs = synth.Ligands.from_parts([one, rigid, empty_move, chain])
    orient = synth.orientations(1, 3)
    res = dock.dock_batch_hybrid(h, ligs, orient, 16, cpu_threads=2, use_gpu=False, want_all=True)
    rep = check_batch(p, ligs, orient, 16, res)
    assert rep.ok(), rep.summary()
    ref = oracle.dock_batch(p, ligs, orient, 16)
    assert np.array_equal(res["best_orient"], ref.best_orient)


def test_hybrid_splits_one_batch_between_gpu_and_host(pockets):
    """GPU chunks and host threads from one dispenser: every ligand docked
    once; the GPU's ligands equal dock_batch bit for bit; the host's pass
    the reference check."""
    p, h = pockets(3)
    ligs = synth.ligands(3, count=1500, first=2000)
    orient = synth.orientations(3, 16)
    S = 128
    print(f"[hybrid] GPU + 6 host threads: {ligs.n_ligands} ligands x 16 orientations", flush=True)
    res = dock.dock_batch_hybrid(h, ligs, orient, S, cpu_threads=6, gpu_chunk=200, cpu_chunk=2,
                                 want_all=True)
    st = res["stats"]
    print(st, flush=True)
    assert set(np.unique(res["done_by"]).tolist()) <= {0, 1}
    assert st["gpu_ligands"] + st["cpu_ligands"] == ligs.n_ligands
    assert st["gpu_ligands"] == int((res["done_by"] == 0).sum()) > 0
    assert st["cpu_ligands"] == int((res["done_by"] == 1).sum()) > 0
    assert st["gpu_chunks"] >= 2
    assert (res["status"] == 0).all()
    ref = dock.dock_batch(h, ligs, orient, S, want_all=True)
    gpu = np.flatnonzero(res["done_by"] == 0)
    for l in gpu:
        for k in ("best_score", "best_orient", "all_scores"):
            assert np.array_equal(res[k][l], ref[k][l]), (k, l)
        a0, a1 = ligs.atom_offset[l], ligs.atom_offset[l + 1]
        assert np.array_equal(res["xyz"][a0:a1], ref["xyz"][a0:a1])
        r0, r1 = ligs.rot_offset[l], ligs.rot_offset[l + 1]
        assert np.array_equal(res["angle_idx"][r0:r1], ref["angle_idx"][r0:r1])
        assert np.array_equal(res["all_angle_idx"][r0 * 16:r1 * 16], ref["all_angle_idx"][r0 * 16:r1 * 16])
    host = np.flatnonzero(res["done_by"] == 1)
    rng = np.random.default_rng(3)
    pick = rng.choice(host, min(40, len(host)), replace=False)
    rep = check_batch(p, ligs, orient, S, res, ligands=pick, orients=[0, 5, 11])
    print(rep.summary())
    assert rep.ok(), rep.summary()
    rep.assert_rare()


def test_hybrid_gpu_only_matches_sync(pockets):
    """use_gpu with no host threads: the pipelined chunks equal dock_batch."""
    p, h = pockets(2)
    ligs = synth.ligands(2, count=700, first=3000)
    orient = synth.orientations(2, 32)
    res = dock.dock_batch_hybrid(h, ligs, orient, 256, cpu_threads=0, gpu_chunk=150)
    ref = dock.dock_batch(h, ligs, orient, 256)
    assert (res["done_by"] == 0).all() and res["stats"]["gpu_chunks"] >= 5
    for k in ("best_score", "best_orient", "angle_idx", "xyz"):
        assert np.array_equal(res[k], ref[k]), k


def test_hybrid_refusals(pockets):
    p, h = pockets(1)
    ligs, orient = synth.ligands(1), synth.orientations(1)
    for kw in (dict(use_gpu=False, cpu_threads=0), dict(mode=dock.DOCK_MODE_LEARNED),
               dict(align=np.eye(3, dtype=np.float32)[None])):
        with pytest.raises(dock.DockError) as e:
            dock.dock_batch_hybrid(h, ligs, orient, 64, **kw)
        assert e.value.code == dock.DOCK_E_INVAL, kw
