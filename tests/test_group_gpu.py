"""Grouped mapping of the plain sweep (dock_set_group_mapping): several
orientations of one small ligand per wave in 16- or 32-lane groups.

Results must be bitwise those of the one-item-per-wave mapping on every
output, whatever the class bounds; the grouped runs are also replayed by the
FP64 reference like every other GPU result.
"""
import numpy as np
import pytest

from paper_1901_06229_amd import dock, synth
from tests.checker import check_batch

pytestmark = pytest.mark.gpu

NAMES = ("best_score", "best_orient", "angle_idx", "xyz", "all_scores", "all_angle_idx", "status")
MAPPINGS = [(0, 0), (32, 64), (40, 80), (48, 96), (64, 128), (80, 128), (96, 128), (80, 192), (0, 160),
            (0, 96), (48, 0)]


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
        dock.dock_set_group_mapping(h, 0, 0)
        h.close()


def _run(h, ligs, orient, S, mapping, split=0, **kw):
    dock.dock_set_group_mapping(h, *mapping)
    dock.dock_set_group_split(h, split)
    print(f"[group] mapping {mapping} split {split}: {ligs.n_ligands} ligands x "
          f"{orient.shape[0]} orientations, S={S} {kw}", flush=True)
    return dock.dock_batch(h, ligs, orient, S, want_all=True, **kw)


def _same(a, b, what):
    for k in NAMES:
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), (what, k)


def test_grouped_results_are_bitwise_the_single_item_ones(pockets):
    """Uneven ligands (8-150 atoms), an orientation count that leaves idle
    groups in a ligand's last wave (22 = 5 x 4 + 2), every class bound."""
    p, h = pockets(3)
    ligs = synth.ligands(3, count=400, first=300)
    orient = synth.orientations(3, 22)
    ref = _run(h, ligs, orient, 128, (0, 0))
    for mp in MAPPINGS[1:]:
        _same(_run(h, ligs, orient, 128, mp), ref, mp)
    # the 32-lane ligands in classes of 32, 48 or 64 atoms (up to 6 of them),
    # and widths that leave one class
    for mp, split in (((64, 160), 32), ((48, 150), 48), ((0, 192), 32), ((0, 128), 64),
                      ((64, 128), 64), ((64, 128), 128)):
        _same(_run(h, ligs, orient, 128, mp, split), ref, (mp, split))


@pytest.mark.parametrize("S", [1, 7, 16, 17, 33, 127, 128, 129, 255, 257, 360, 2048])
def test_grouped_step_counts(pockets, S):
    """Step counts around the 16- and 32-step tiles, the 32- and 64-step
    compaction chunks, the rings of 64 and 128 compacted steps, the 32-bit
    mask words and the largest step count the grouped mapping takes."""
    p, h = pockets(2)
    ligs = synth.ligands(2, count=24, first=900)
    orient = synth.orientations(2, 9)
    ref = _run(h, ligs, orient, S, (0, 0))
    got = _run(h, ligs, orient, S, (80, 128))
    _same(got, ref, S)


def test_grouped_parity_with_reference(pockets):
    """Grouped runs replayed item by item by the FP64 reference."""
    p, h = pockets(3)
    ligs = synth.ligands(3, count=60, first=4000)
    orient = synth.orientations(3, 12)
    res = _run(h, ligs, orient, 128, (48, 96))
    rep = check_batch(p, ligs, orient, 128, res, orients=[0, 3, 7, 11])
    print(rep.summary())
    assert rep.ok(), rep.summary()
    rep.assert_rare()
    p1, h1 = pockets(1)
    res = _run(h1, synth.ligands(1), synth.orientations(1), 64, (64, 0))
    rep = check_batch(p1, synth.ligands(1), synth.orientations(1), 64, res)
    assert rep.ok(), rep.summary()


def test_grouped_passes_and_class_limits(pockets):
    """Two passes, and ligands at exactly the class bounds (64, 80 and 96
    atoms in the 16-lane class, 128 and 150 in the 32-lane class), next to
    larger ones."""
    p, h = pockets(3)
    all_ligs = synth.ligands(3, count=3000)
    n = np.diff(all_ligs.atom_offset)
    pick = []
    for lo, hi in ((60, 64), (76, 80), (92, 96), (120, 128), (129, 150), (8, 20)):
        pick += list(np.flatnonzero((n >= lo) & (n <= hi))[:4])
    ligs = all_ligs.subset(pick)
    print("atoms", np.diff(ligs.atom_offset).tolist(), flush=True)
    orient = synth.orientations(3, 10)
    ref = _run(h, ligs, orient, 128, (0, 0), passes=2)
    for mp in ((64, 128), (80, 128), (96, 128), (80, 150), (64, 192)):
        _same(_run(h, ligs, orient, 128, mp, passes=2), ref, ("passes 2", mp))
    rep = check_batch(p, ligs, orient, 128, _run(h, ligs, orient, 128, (80, 192), passes=2),
                      passes=2, orients=[0, 9])
    assert rep.ok(), rep.summary()


def test_grouped_large_ligands(pockets):
    """The 32-lane class up to its 192-atom limit on the large-ligand pocket
    (256^3 grid, 360 steps, 60-120 rotamers): ligands of 100-192 atoms, with
    one at or next to each bound, bitwise equal to one item per wave."""
    p, h = pockets(5)
    all_ligs = synth.ligands(5, count=400)
    n = np.diff(all_ligs.atom_offset)
    pick = []
    for lo, hi in ((100, 128), (129, 160), (180, 192), (193, 250)):
        pick += list(np.flatnonzero((n >= lo) & (n <= hi))[:3])
    ligs = all_ligs.subset(pick)
    print("atoms", np.diff(ligs.atom_offset).tolist(), flush=True)
    orient = synth.orientations(5, 4)
    ref = _run(h, ligs, orient, 360, (0, 0))
    for mp in ((80, 192), (0, 160), (64, 128)):
        _same(_run(h, ligs, orient, 360, mp), ref, mp)
    for mp, split in (((80, 192), 48), ((80, 192), 32), ((0, 192), 150)):
        _same(_run(h, ligs, orient, 360, mp, split), ref, (mp, split))


def test_grouped_async_graph_replay(pockets):
    """Device-array calls, eager and as a replayed HIP graph, with the grouped
    mapping (one 32-lane class, and the 32-lane ligands in classes 32 atoms
    wide, the launch the bench replays): equal to the synchronous
    one-item-per-wave call."""
    import torch
    from tests.test_parity_gpu import _device_batch
    p, h = pockets(3)
    ligs = synth.ligands(3, count=500, first=7000)
    orient = synth.orientations(3, 16)
    ref = _run(h, ligs, orient, 128, (0, 0))
    d, od, out = _device_batch(ligs, orient, 128, torch)
    ws = torch.empty(dock.dock_workspace_size(ligs.n_ligands, d["total_rot"], 16, 128),
                     dtype=torch.uint8, device="cuda:0")
    st = torch.cuda.Stream()
    mx = int(np.diff(ligs.atom_offset).max())
    names = NAMES[:-1]
    for mp, split in (((40, 80), 0), ((64, 192), 32)):
        dock.dock_set_group_mapping(h, *mp)
        dock.dock_set_group_split(h, split)
        for flags in (0, dock.DOCK_FLAG_GRAPH, dock.DOCK_FLAG_GRAPH):
            for k in names:
                out[k].fill_(0)
            torch.cuda.synchronize()
            dock.dock_batch_async(h, d, od, 128, out, dock.make_params(max_atoms=mx, flags=flags),
                                  workspace=ws, stream=st)
            st.synchronize()
            got = {k: out[k].cpu().numpy() for k in names}
            got["xyz"] = got["xyz"].reshape(-1, 3)
            for k in names:
                assert np.array_equal(np.asarray(ref[k]).reshape(got[k].shape), got[k]), \
                    (mp, split, flags, k)
    dock.dock_set_group_split(h, 0)


def test_group_mapping_arguments(pockets):
    p, h = pockets(1)
    for a, b, code in ((97, 0, dock.DOCK_E_LIMIT), (0, 193, dock.DOCK_E_LIMIT),
                       (48, 40, dock.DOCK_E_INVAL), (-1, 0, dock.DOCK_E_LIMIT)):
        with pytest.raises(dock.DockError) as e:
            dock.dock_set_group_mapping(h, a, b)
        assert e.value.code == code
    dock.dock_set_group_mapping(h, 32, 64)
    assert dock.dock_get_group_mapping(h) == (32, 64)
    dock.dock_set_group_mapping(h, 0, 0)
    for bad in (-1, 16, 31, 193):
        with pytest.raises(dock.DockError) as e:
            dock.dock_set_group_split(h, bad)
        assert e.value.code == dock.DOCK_E_LIMIT
    dock.dock_set_group_split(h, 32)
    assert dock.dock_get_group_split(h) == 32
    dock.dock_set_group_split(h, 0)
    assert dock.dock_get_group_split(h) == 0


def test_grouped_degenerate_ligands(pockets):
    """One atom, no rotamers, an empty moving set, a three-atom chain and a
    whole ligand, with 1 and 5 orientations (3 or 3 + 3 idle groups per
    wave), bitwise equal to the one-item-per-wave mapping; the r_bump = 50
    case where no angle is valid (k* = -1 everywhere) too."""
    from tests.helpers import make_lig
    p, h = pockets(1)
    one = make_lig(np.array([[0.5, 0.2, -0.3]], np.float32), [])
    xyz = np.array([[0, 0, 0], [1.5, 0, 0], [2.0, 1.4, 0], [3.5, 1.5, 0.3]], np.float32)
    rigid = make_lig(xyz, [])
    empty_move = make_lig(xyz, [(0, 1, [])])
    chain = make_lig(xyz, [(1, 2, [3])])
    whole = synth.ligands(1).ligand(0)
    ligs = synth.Ligands.from_parts([one, rigid, empty_move, chain, whole])
    for O in (1, 5):
        orient = synth.orientations(1, O)
        for S in (1, 16, 100):
            ref = _run(h, ligs, orient, S, (0, 0))
            for mp in ((80, 128), (0, 128)):
                _same(_run(h, ligs, orient, S, mp), ref, (O, S, mp))
        ref = _run(h, ligs, orient, 16, (0, 0), r_bump=50.0)
        got = _run(h, ligs, orient, 16, (80, 128), r_bump=50.0)
        _same(got, ref, (O, "r_bump 50"))
        # every rotamer with moving atoms bumps at every angle; the one with
        # an empty moving set (the first rotamer of the batch) cannot bump
        ai = np.asarray(got["angle_idx"]).reshape(-1)
        assert ai[0] == 0 and (ai[1:] == -1).all(), ai
