"""GPU sweep vs the FP64 reference through the C-ABI (libdock.so).

Every item (ligand x orientation) checked here is replayed by the reference
along the GPU's own angle choices (tests/checker.py): the bar is 1e-4 A on
coordinates, 1e-5 relative on scores and the same angle indices except at
reference gaps below 1e-5 or at recorded FP32/FP64 ambiguities.
"""
import numpy as np
import pytest

import oracle
from paper_1901_06229_amd import dock, synth
from tests.checker import check_batch, tol_of

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


def _run(pockets, cfg, ligs, orient, S, **kw):
    p, h = pockets(cfg)
    print(f"[gpu] config {cfg}: {ligs.n_ligands} ligands x {orient.shape[0]} orientations, S={S}",
          flush=True)
    res = dock.dock_batch(h, ligs, orient, S, want_all=True, **kw)
    return p, res


def test_c1_parity(pockets):
    ligs = synth.ligands(1)
    orient = synth.orientations(1)
    p, res = _run(pockets, 1, ligs, orient, 64)
    rep = check_batch(p, ligs, orient, 64, res)
    print(rep.summary())
    assert rep.ok(), rep.summary()
    rep.assert_rare()
    ref = oracle.dock_batch(p, ligs, orient, 64)
    assert abs(res["best_score"][0] - ref.best_score[0]) <= tol_of(ref.best_score[0])
    assert np.abs(res["all_scores"] - ref.all_scores).max() <= tol_of(np.abs(ref.all_scores).max())
    assert (res["status"] == 0).all()


def test_c2_subset_parity(pockets):
    """C2 shapes (128^3 pocket, 256 orientations, 256 steps) on 200 ligands:
    every orientation of 6 ligands, 8 sampled orientations of all 200."""
    ligs = synth.ligands(2, count=200)
    orient = synth.orientations(2)
    p, res = _run(pockets, 2, ligs, orient, 256)
    assert (res["status"] == 0).all()
    rep = check_batch(p, ligs, orient, 256, res, ligands=range(6))
    print(rep.summary())
    assert rep.ok(), rep.summary()
    rep.assert_rare()
    rng = np.random.default_rng(0)
    rep2 = check_batch(p, ligs, orient, 256, res, ligands=range(200),
                       orients=rng.choice(256, 8, replace=False))
    print(rep2.summary())
    assert rep2.ok(), rep2.summary()
    rep2.assert_rare()
    amb = rep2.steps["ambiguous"] / max(1, sum(rep2.steps.values()))
    assert amb < 0.01


def test_c3_subset_parity(pockets):
    """C3 shapes (lognormal sizes 8-150, 0-40 rotamers, 128 orientations, 128 steps)."""
    ligs = synth.ligands(3, count=300)
    orient = synth.orientations(3)
    p, res = _run(pockets, 3, ligs, orient, 128)
    rng = np.random.default_rng(1)
    rep = check_batch(p, ligs, orient, 128, res, ligands=range(300),
                      orients=rng.choice(128, 4, replace=False))
    print(rep.summary())
    assert rep.ok(), rep.summary()
    rep.assert_rare()


def test_c5_subset_parity(pockets):
    """C5 shapes (256^3 irregular pocket, 100-250 atoms, 60-120 rotamers, 360 steps)."""
    ligs = synth.ligands(5, count=12)
    orient = synth.orientations(5)
    p, res = _run(pockets, 5, ligs, orient, 360)
    rng = np.random.default_rng(2)
    rep = check_batch(p, ligs, orient, 360, res, ligands=range(12),
                      orients=rng.choice(64, 2, replace=False))
    print(rep.summary())
    assert rep.ok(), rep.summary()
    rep.assert_rare()


def test_full_c2_batch_in_bench_configuration(pockets):
    """The C2 batch at full size (10,000 ligands x 256 orientations x 256
    steps) under the launch bench.py times (automatic block size, claim cap 16):
    items sampled across the cost-sorted queue are replayed by the reference
    one by one, and every ligand's winner is the best of its 256 orientation
    scores with the lowest index on ties."""
    p, h = pockets(2)
    ligs = synth.ligands(2)
    assert ligs.n_ligands == 10_000
    orient = synth.orientations(2)
    dock.dock_set_launch(h, 0, 0, 16)
    res = _run(pockets, 2, ligs, orient, 256)[1]
    assert (res["status"] == 0).all()
    sc = res["all_scores"]
    best = sc.max(axis=1)
    assert np.array_equal(res["best_score"], best)
    assert np.array_equal(res["best_orient"], np.argmax(sc == best[:, None], axis=1))
    rng = np.random.default_rng(11)
    sample = rng.choice(ligs.n_ligands, 16, replace=False)
    rep = check_batch(p, ligs, orient, 256, res, ligands=sample,
                      orients=rng.choice(256, 3, replace=False))
    print(rep.summary())
    assert rep.ok(), rep.summary()
    rep.assert_rare()


def test_determinism_and_order_independence(pockets):
    ligs = synth.ligands(2, count=300, first=1000)
    orient = synth.orientations(2, 64)
    p, a = _run(pockets, 2, ligs, orient, 128)
    _, b = _run(pockets, 2, ligs, orient, 128)
    _, c = _run(pockets, 2, ligs, orient, 128, flags=dock.DOCK_FLAG_NO_LPT)
    for k in ("best_score", "best_orient", "angle_idx", "xyz", "all_scores", "all_angle_idx"):
        assert np.array_equal(a[k], b[k]), k
        assert np.array_equal(a[k], c[k]), k


def test_edge_cases(pockets):
    p, h = pockets(1)
    base = synth.ligands(1)
    lig = base.ligand(0)
    n = len(lig["xyz"])
    no_rot = dict(xyz=lig["xyz"], rot_axis=np.zeros((0, 2), np.int32),
                  move_offset=np.zeros(1, np.int32), move_atoms=np.zeros(0, np.int16))
    one_atom = dict(xyz=lig["xyz"][:1], rot_axis=np.zeros((0, 2), np.int32),
                    move_offset=np.zeros(1, np.int32), move_atoms=np.zeros(0, np.int16))
    ligs = synth.Ligands.from_parts([lig, no_rot, one_atom, lig])
    orient = synth.orientations(1, 3)
    for S in (1, 2, 63, 64, 65, 200, dock.DOCK_MAX_STEPS):
        res = dock.dock_batch(h, ligs, orient, S, want_all=True)
        rep = check_batch(p, ligs, orient, S, res)
        assert rep.ok(), (S, rep.summary())
        rep.assert_rare()
        assert np.array_equal(res["best_score"][0], res["best_score"][3])
    # a bump radius so large that no angle (not even k = 0) is valid: k* = -1, no move
    res = dock.dock_batch(h, ligs, orient, 16, r_bump=50.0, want_all=True)
    assert (res["angle_idx"] == -1).all()
    rep = check_batch(p, ligs, orient, 16, res, r_bump=50.0)
    assert rep.ok(), rep.summary()
    rep.assert_rare()
    # empty batch
    empty = synth.Ligands.from_parts([])
    res = dock.dock_batch(h, empty, orient, 16)
    assert res["best_score"].shape == (0,)


@pytest.mark.parametrize("S", [3, 5, 7, 31, 32, 33, 95, 97, 360])
def test_step_counts_around_mask_words(pockets, S):
    """Clash arcs are marked 32 steps to a bitmask word, an arc that wraps past
    step S - 1 as two ranges: step counts below, at and just past word and
    tile boundaries, on 24 ligands of 20-80 atoms (128^3 pocket) x 16
    orientations, every item replayed by the reference."""
    p, h = pockets(2)
    ligs = synth.ligands(2, count=24, first=7000)
    orient = synth.orientations(2, 16)
    print(f"[gpu] step counts: 24 ligands x 16 orientations, S={S}", flush=True)
    res = dock.dock_batch(h, ligs, orient, S, want_all=True)
    assert (res["status"] == 0).all()
    rep = check_batch(p, ligs, orient, S, res)
    print(rep.summary())
    assert rep.ok(), (S, rep.summary())
    rep.assert_rare()


def test_max_size_ligand(pockets):
    """A 256-atom ligand (the per-ligand maximum) with 255 rotamers."""
    p, h = pockets(5)
    big = synth.ligands(5, count=40)
    l = int(np.argmax(np.diff(big.atom_offset)))
    lig = big.ligand(l)
    n = len(lig["xyz"])
    # pad to 256 atoms with far-away isolated atoms and repeat rotamers up to 255
    extra = 256 - n
    far = np.stack([np.array([30.0, 30.0, 30.0]) + 3.0 * np.array([i % 6, (i // 6) % 6, i // 36])
                    for i in range(extra)]).astype(np.float32)
    R = len(lig["rot_axis"])
    reps = [r % R for r in range(255)]
    moff = [0]
    mv = []
    for r in reps:
        seg = lig["move_atoms"][lig["move_offset"][r]:lig["move_offset"][r + 1]]
        mv.extend(seg.tolist())
        moff.append(len(mv))
    big_lig = dict(xyz=np.concatenate([lig["xyz"], far]), rot_axis=lig["rot_axis"][reps],
                   move_offset=np.asarray(moff, np.int32), move_atoms=np.asarray(mv, np.int16))
    ligs = synth.Ligands.from_parts([big_lig])
    orient = synth.orientations(5, 2)
    res = dock.dock_batch(h, ligs, orient, 32, want_all=True)
    rep = check_batch(p, ligs, orient, 32, res)
    print(rep.summary())
    assert rep.ok(), rep.summary()
    rep.assert_rare()


def test_passes_refinement(pockets):
    """num_repetitions > 1 (paper Listing 1): the sweep over all rotamers repeats."""
    p, res = None, None
    ligs = synth.ligands(2, count=20, first=50)
    orient = synth.orientations(2, 8)
    p, res = _run(pockets, 2, ligs, orient, 64, passes=3)
    rep = check_batch(p, ligs, orient, 64, res, passes=3)
    print(rep.summary())
    assert rep.ok(), rep.summary()
    rep.assert_rare()


def test_invalid_inputs_rejected_before_launch(pockets):
    p, h = pockets(1)
    lig = synth.ligands(1).ligand(0)
    bad = dict(lig)
    bad["move_atoms"] = lig["move_atoms"].copy()
    bad["move_atoms"][0] = 99
    ligs = synth.Ligands.from_parts([bad])
    with pytest.raises(dock.DockError) as e:
        dock.dock_batch(h, ligs, synth.orientations(1), 16)
    assert e.value.code == dock.DOCK_E_INVAL
    with pytest.raises(dock.DockError) as e:
        dock.dock_batch(h, synth.ligands(1), synth.orientations(1), 5000)
    assert e.value.code == dock.DOCK_E_LIMIT


def test_direct_bump_mode_parity(pockets):
    """The literal form (every cross pair tested at every angle) on the same
    inputs, checked against the reference like the default kernel."""
    ligs = synth.ligands(2, count=40, first=300)
    orient = synth.orientations(2, 32)
    p, res = _run(pockets, 2, ligs, orient, 256, flags=dock.DOCK_FLAG_DIRECT_BUMP)
    rep = check_batch(p, ligs, orient, 256, res, ligands=range(40), orients=range(0, 32, 4))
    print(rep.summary())
    assert rep.ok(), rep.summary()
    rep.assert_rare()
    ligs1 = synth.ligands(1)
    o1 = synth.orientations(1)
    p1, r1 = _run(pockets, 1, ligs1, o1, 64, flags=dock.DOCK_FLAG_DIRECT_BUMP)
    rep = check_batch(p1, ligs1, o1, 64, r1)
    assert rep.ok(), rep.summary()
    rep.assert_rare()


def test_results_independent_of_launch_mapping(pockets):
    """Bitwise-identical results for every waves-per-block / blocks-per-CU /
    claim-cap plan (claims shrink to single items at the end of the queue)."""
    p, h = pockets(2)
    ligs = synth.ligands(2, count=150, first=2000)
    orient = synth.orientations(2, 32)
    ref = None
    for waves, bpc, claim in ((4, 0, 1), (1, 0, 1), (2, 1, 4), (4, 2, 8), (1, 3, 64), (4, 0, 3),
                              (0, 0, 32), (0, 0, 16)):
        dock.dock_set_launch(h, waves, bpc, claim)
        res = dock.dock_batch(h, ligs, orient, 128, want_all=True)
        if ref is None:
            ref = res
            continue
        for k in ("best_score", "best_orient", "angle_idx", "xyz", "all_scores", "all_angle_idx"):
            assert np.array_equal(ref[k], res[k]), (waves, bpc, claim, k)
    dock.dock_set_launch(h, 0, 0, 16)


def test_autotune_picks_fastest_and_keeps_results(pockets):
    p, h = pockets(2)
    ligs = synth.ligands(2, count=400, first=3000)
    orient = synth.orientations(2, 64)
    before = dock.dock_batch(h, ligs, orient, 128, want_all=True)
    entries = dock.dock_autotune(h, ligs, orient, 128, sample_ligands=100, seed=7)
    print(entries)
    # waves {0, 1, 2, 4} x claim caps {4, 16, 32, 64} x six group bounds and splits
    assert len(entries) == 96
    best = min(entries, key=lambda e: e["sweep_ms"])
    assert dock.dock_get_launch(h) == (best["waves_per_block"], best["blocks_per_cu"],
                                       best["items_per_claim"])
    assert dock.dock_get_group_mapping(h) == (best["group16_atoms"], best["group32_atoms"])
    assert dock.dock_get_group_split(h) == best["group32_split"]
    after = dock.dock_batch(h, ligs, orient, 128, want_all=True)
    for k in ("best_score", "best_orient", "angle_idx", "xyz", "all_scores", "all_angle_idx"):
        assert np.array_equal(before[k], after[k]), k
    dock.dock_set_launch(h, 0, 0, 16)
    dock.dock_set_group_mapping(h, 80, 192)
    dock.dock_set_group_split(h, 0)


def _device_batch(ligs, orient, S, torch):
    dev = torch.device("cuda:0")
    d = dict(n_ligands=ligs.n_ligands, total_atoms=int(ligs.atom_offset[-1]),
             total_rot=int(ligs.rot_offset[-1]), total_move=int(ligs.move_offset[-1]))
    for k, dt in (("atom_offset", torch.int32), ("xyz", torch.float32), ("rot_offset", torch.int32),
                  ("rot_axis", torch.int32), ("move_offset", torch.int32), ("move_atoms", torch.int16)):
        d[k] = torch.from_numpy(np.ascontiguousarray(getattr(ligs, k))).to(dev, dt)
    L, NA, NR = ligs.n_ligands, d["total_atoms"], d["total_rot"]
    out = dict(best_score=torch.empty(L, device=dev),
               best_orient=torch.empty(L, dtype=torch.int32, device=dev),
               angle_idx=torch.empty(NR, dtype=torch.int16, device=dev),
               xyz=torch.empty(NA, 3, device=dev), status=torch.empty(L, dtype=torch.int32, device=dev),
               all_scores=torch.empty(L, orient.shape[0], device=dev),
               all_angle_idx=torch.empty(NR * orient.shape[0], dtype=torch.int16, device=dev))
    return d, torch.from_numpy(orient).to(dev), out


def test_graph_replay_with_sweep_timing(pockets):
    """The benchmark's uneven-batch mode: a replayed HIP graph that also records
    the sweep's timing events and work counters.  Every replay matches the
    eager call and reports its own kernel time and counters."""
    import torch
    p, h = pockets(2)
    ligs = synth.ligands(3, count=300, first=100)
    orient = synth.orientations(2, 16)
    d, od, out = _device_batch(ligs, orient, 128, torch)
    ws = torch.empty(dock.dock_workspace_size(ligs.n_ligands, d["total_rot"], 16, 128),
                     dtype=torch.uint8, device="cuda:0")
    st = torch.cuda.Stream()
    mx = int(np.diff(ligs.atom_offset).max())
    names = ("best_score", "best_orient", "angle_idx", "xyz", "all_scores", "all_angle_idx")
    eager = dock.make_params(max_atoms=mx, flags=dock.DOCK_FLAG_TIME_SWEEP)
    for _ in range(2):  # the first launch also loads the kernels' code
        dock.dock_batch_async(h, d, od, 128, out, eager, workspace=ws, stream=st)
    st.synchronize()
    ref = {k: out[k].cpu().numpy() for k in names}
    ref_work = dock.dock_last_sweep_work(h)
    sweep_ms = dock.dock_last_sweep_ms(h)
    gprm = dock.make_params(max_atoms=mx, flags=dock.DOCK_FLAG_TIME_SWEEP | dock.DOCK_FLAG_GRAPH)
    for _ in range(3):
        for k in names:
            out[k].fill_(0)
        torch.cuda.synchronize()
        dock.dock_batch_async(h, d, od, 128, out, gprm, workspace=ws, stream=st)
        ms = dock.dock_last_sweep_ms(h)
        # the replayed graph is timed as a whole: the sweep dominates it
        assert 0.9 * sweep_ms <= ms <= 1.5 * sweep_ms + 0.5, (ms, sweep_ms)
        assert dock.dock_last_sweep_work(h) == ref_work
        st.synchronize()
        for k in names:
            assert np.array_equal(ref[k], out[k].cpu().numpy()), k


def test_sweep_ms_history():
    """Timed calls enqueued back to back, read afterwards: the handle keeps the
    sweep events of its last 16 timed calls, oldest first, the last equal to
    dock_last_sweep_ms; asking for more than were made, or than it keeps, fails.
    A fresh handle, so no earlier timed call is on it."""
    import torch
    pocket = synth.pocket(2)
    h = dock.dock_init_pocket(pocket.grid, pocket.origin, pocket.spacing)
    try:
        ligs = synth.ligands(2, count=40, first=3000)
        orient = synth.orientations(2, 8)
        d, od, out = _device_batch(ligs, orient, 64, torch)
        ws = torch.empty(dock.dock_workspace_size(ligs.n_ligands, d["total_rot"], 8, 64),
                         dtype=torch.uint8, device="cuda:0")
        st = torch.cuda.Stream()
        prm = dock.make_params(max_atoms=int(np.diff(ligs.atom_offset).max()),
                               flags=dock.DOCK_FLAG_TIME_SWEEP)
        with pytest.raises(dock.DockError) as e:
            dock.dock_sweep_ms_history(h, 1)
        assert e.value.code == dock.DOCK_E_STATE
        for _ in range(3):
            dock.dock_batch_async(h, d, od, 64, out, prm, workspace=ws, stream=st)
        ms = dock.dock_sweep_ms_history(h, 3)
        assert len(ms) == 3 and all(0.0 < x < 1e4 for x in ms), ms
        assert ms[-1] == dock.dock_last_sweep_ms(h)
        with pytest.raises(dock.DockError) as e:
            dock.dock_sweep_ms_history(h, 4)
        assert e.value.code == dock.DOCK_E_STATE
        for _ in range(17):  # wraps the ring
            dock.dock_batch_async(h, d, od, 64, out, prm, workspace=ws, stream=st)
        ms = dock.dock_sweep_ms_history(h, 16)
        assert len(ms) == 16 and all(0.0 < x < 1e4 for x in ms), ms
        assert ms[-1] == dock.dock_last_sweep_ms(h)
        for bad in (0, 17):
            with pytest.raises(dock.DockError) as e:
                dock.dock_sweep_ms_history(h, bad)
            assert e.value.code == dock.DOCK_E_INVAL
        st.synchronize()
        assert int((out["status"] != 0).sum()) == 0
    finally:
        h.close()


def test_device_validation_codes(pockets):
    """Device-array calls validate every ligand on the device (one wave per
    ligand): malformed ligands get their DOCK_E_* code and best_orient = -1,
    and the valid ligands between them get the synchronous call's results."""
    import torch
    p, h = pockets(2)
    src = synth.ligands(2, count=16, first=4000)
    parts = [src.ligand(i) for i in range(src.n_ligands)]
    mx = max(len(q["xyz"]) for q in parts)
    with_rot = [i for i, q in enumerate(parts) if len(q["move_offset"]) > 2 and
                q["move_offset"][1] - q["move_offset"][0] >= 2]
    i0, i1, i2 = with_rot[:3]
    out_of_range = dict(parts[i0], move_atoms=parts[i0]["move_atoms"].copy())
    out_of_range["move_atoms"][0] = len(out_of_range["xyz"])          # atom index past n
    same_axis = dict(parts[i1], rot_axis=parts[i1]["rot_axis"].copy())
    same_axis["rot_axis"][0, 1] = same_axis["rot_axis"][0, 0]          # a == b
    unsorted = dict(parts[i2], move_atoms=parts[i2]["move_atoms"].copy())
    m0 = int(unsorted["move_offset"][0])
    unsorted["move_atoms"][[m0, m0 + 1]] = unsorted["move_atoms"][[m0 + 1, m0]]  # not increasing
    reps = -(-(mx + 1) // len(parts[0]["xyz"]))
    big = dict(xyz=np.tile(parts[0]["xyz"], (reps, 1))[:mx + 1], rot_axis=np.zeros((0, 2), np.int32),
               move_offset=np.zeros(1, np.int32), move_atoms=np.zeros(0, np.int16))  # n > max_atoms
    good = [parts[j] for j in range(len(parts)) if j not in (i0, i1, i2)][:4]
    batch = [good[0], out_of_range, good[1], same_axis, good[2], unsorted, big, good[3]]
    want = [0, dock.DOCK_E_INVAL, 0, dock.DOCK_E_INVAL, 0, dock.DOCK_E_INVAL, dock.DOCK_E_LIMIT, 0]
    ligs = synth.Ligands.from_parts(batch)
    orient = synth.orientations(2, 8)
    d, od, out = _device_batch(ligs, orient, 64, torch)
    st = torch.cuda.Stream()
    print("[gpu] device validation: 8 ligands, 4 malformed", flush=True)
    dock.dock_batch_async(h, d, od, 64, out, dock.make_params(max_atoms=mx), stream=st)
    st.synchronize()
    assert out["status"].cpu().tolist() == want
    best_orient = out["best_orient"].cpu().numpy()
    assert (best_orient[[1, 3, 5, 6]] == -1).all()
    ref = dock.dock_batch(h, synth.Ligands.from_parts(good), orient, 64, want_all=True)
    rows = [0, 2, 4, 7]
    assert np.array_equal(out["best_score"].cpu().numpy()[rows], ref["best_score"])
    assert np.array_equal(best_orient[rows], ref["best_orient"])
    assert np.array_equal(out["all_scores"].cpu().numpy()[rows], ref["all_scores"])


def test_async_rejects_host_memory(pockets):
    """Pageable host arrays passed to the device-array entry point are refused
    on the host before anything is enqueued.  The workspace is also too small,
    so even a missed check would stop before any launch."""
    import torch
    p, h = pockets(2)
    ligs = synth.ligands(2, count=8, first=300)
    orient = synth.orientations(2, 4)
    d, od, out = _device_batch(ligs, orient, 32, torch)
    tiny = torch.empty(256, dtype=torch.uint8, device="cuda:0")
    prm = dock.make_params(max_atoms=int(np.diff(ligs.atom_offset).max()))
    with pytest.raises(dock.DockError) as e:
        dock.dock_batch_async(h, d, torch.from_numpy(orient), 32, out, prm, workspace=tiny)
    assert e.value.code == dock.DOCK_E_INVAL and "orient is not device-accessible" in str(e.value)
    host_rot = torch.from_numpy(synth.align_rotations(2, 4))
    with pytest.raises(dock.DockError) as e:
        dock.dock_batch_async(h, d, od, 32, out, dock.make_params(align=host_rot), workspace=tiny)
    assert "align_rot is not device-accessible" in str(e.value)
    bad_out = dict(out, xyz=torch.empty(int(ligs.atom_offset[-1]), 3))
    with pytest.raises(dock.DockError) as e:
        dock.dock_batch_async(h, d, od, 32, bad_out, prm, workspace=tiny)
    assert "xyz_out is not device-accessible" in str(e.value)
    # with device arrays the same call fails only on the workspace size
    with pytest.raises(dock.DockError) as e:
        dock.dock_batch_async(h, d, od, 32, out, prm, workspace=tiny)
    assert "workspace too small" in str(e.value)
    torch.cuda.synchronize()


def test_async_and_graph_replay_match_sync(pockets):
    """dock_batch_async on device tensors, eager and as a replayed HIP graph
    (several replays with eager work and synchronisation in between), against
    the synchronous host-array call."""
    import torch
    p, h = pockets(2)
    ligs = synth.ligands(2, count=120, first=4000)
    orient = synth.orientations(2, 32)
    ref = dock.dock_batch(h, ligs, orient, 128, want_all=True)
    d, od, out = _device_batch(ligs, orient, 128, torch)
    ws = torch.empty(dock.dock_workspace_size(ligs.n_ligands, d["total_rot"], 32, 128),
                     dtype=torch.uint8, device="cuda:0")
    st = torch.cuda.Stream()
    names = ("best_score", "best_orient", "angle_idx", "xyz", "all_scores", "all_angle_idx")

    def check():
        st.synchronize()
        got = {k: out[k].cpu().numpy() for k in names}
        got["xyz"] = got["xyz"].reshape(-1, 3)
        for k in names:
            assert np.array_equal(np.asarray(ref[k]).reshape(got[k].shape), got[k]), k
        for k in names:
            out[k].fill_(0)
        torch.cuda.synchronize()

    prm = dock.make_params(max_atoms=int(np.diff(ligs.atom_offset).max()))
    dock.dock_batch_async(h, d, od, 128, out, prm, workspace=ws, stream=st)
    check()
    gprm = dock.make_params(max_atoms=int(np.diff(ligs.atom_offset).max()), flags=dock.DOCK_FLAG_GRAPH)
    for rep in range(4):
        dock.dock_batch_async(h, d, od, 128, out, gprm, workspace=ws, stream=st)
        check()
        # unrelated eager work between replays
        x = torch.randn(1000, 1000, device="cuda:0")
        (x @ x).sum().item()


def test_full_c3_batch_autotuned_graph_sampled_replay(pockets):
    """The whole uneven batch (100,000 ligands x 128 orientations x 128 steps)
    as the benchmark runs it: autotuned launch, replayed HIP graph.  Sampled
    items are replayed by the reference; every ligand's best orientation is
    its own argmax; the result equals an eager launch's."""
    import torch
    p, h = pockets(3)
    ligs = synth.ligands(3)
    orient = synth.orientations(3)
    L, O, S = ligs.n_ligands, 128, 128
    tune = dock.dock_autotune(h, ligs, orient, S, sample_ligands=10000, seed=1)
    print(f"[gpu] full uneven batch, autotuned to {dock.dock_get_launch(h)} over {len(tune)} mappings",
          flush=True)
    d, od, out = _device_batch(ligs, orient, S, torch)
    ws = torch.empty(dock.dock_workspace_size(L, d["total_rot"], O, S), dtype=torch.uint8, device="cuda:0")
    st = torch.cuda.Stream()
    mx = int(np.diff(ligs.atom_offset).max())
    names = ("best_score", "best_orient", "angle_idx", "xyz", "all_scores", "all_angle_idx", "status")
    dock.dock_batch_async(h, d, od, S, out, dock.make_params(max_atoms=mx), workspace=ws, stream=st)
    st.synchronize()
    eager = {k: out[k].cpu().numpy() for k in names}
    for k in names:
        out[k].fill_(0)
    torch.cuda.synchronize()
    gprm = dock.make_params(max_atoms=mx, flags=dock.DOCK_FLAG_GRAPH)
    for _ in range(2):  # capture, then a replay
        dock.dock_batch_async(h, d, od, S, out, gprm, workspace=ws, stream=st)
        st.synchronize()
    res = {k: out[k].cpu().numpy() for k in names}
    for k in names:
        assert np.array_equal(res[k], eager[k]), k
    assert (res["status"] == 0).all()
    res["xyz"] = res["xyz"].reshape(-1, 3)
    s = res["all_scores"]
    assert np.array_equal(res["best_orient"], np.argmax(s, axis=1))
    assert np.array_equal(res["best_score"], s[np.arange(L), res["best_orient"]])
    rng = np.random.default_rng(31)
    pick = rng.choice(L, 40, replace=False)
    rep = check_batch(p, ligs, orient, S, res, ligands=pick, orients=rng.choice(O, 2, replace=False))
    print(rep.summary())
    assert rep.ok(), rep.summary()
    rep.assert_rare()
    dock.dock_set_launch(h, 0, 0, 16)
    dock.dock_set_group_mapping(h, 80, 192)
    dock.dock_set_group_split(h, 0)
