"""Throughput benchmark of the batched rotamer sweep on one MI355X.

Headline workload: 100,000 ligands (lognormal 8-150 atoms, 0-40 rotamers) x
128 rigid orientations x 128 angle steps against a 128^3 pocket (synthetic,
seeded), launch mapping autotuned, the launch sequence replayed as a HIP
graph.  Inputs are resident in HBM before the timed region; one step = one
dock_batch_async call over the whole batch (every restart of every ligand,
the per-ligand best reduction and the pose write-back).

Prints one JSON line (rank 0): ligands/s, the sweep kernel's roofline
fraction (HIP events on the kernel's own stream), the synchronous
host-array figure (H2D + kernels + D2H), the FP64 reference timed on bounded
samples on the host cores, and the extra legs under their own keys: the
10,000-ligand batch (c2, with the rigid-alignment leg), the large-ligand
batch (c5, plain and learned proposal side by side, per-ligand error against
the FP64 reference) and the learned-proposal comparison (learned).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ligands/sec on 1 MI355X (plain vs learned proposal at ≤0.5% score loss)"

# MI355X FP32 vector rate: 256 CUs x 128 lanes x 2.4 GHz = 78.6 T lane-ops/s
# (the 157.3 TFLOP/s spec figure, an FMA counted as one lane-op instead of two
# flops).  That rate needs packed FP32 instructions, which this library does
# not use; the VALU probe measures what plain FP32 sustains (about 37 T).
VALU_PEAK_TOPS = 256 * 128 * 2.4e9 / 1e12
# dense BF16 matrix-core rate (published, no sparsity)
MFMA_BF16_PEAK = 2.5e15
# Lane-operation counts (VALU instructions per lane) of the sweep's units,
# taken from the loop bodies of the compiled gfx950 kernels:
#   direct kernel, per angle: 8 per cross pair (3 sub, mul, 2 fma, cmp, or),
#     23 per Rodrigues rotation, 22 per voxel lookup and add
#   pruned kernel, per rotamer step:
#     OPS_CAND per candidate cross pair (m_r q_r of them): 3 lane
#       broadcasts, the cylinder bound (2 sub, mul, fma, cmp) and the append
#       of a kept pair (2 mbcnt on the compare's lane mask, the packed pair
#       and its LDS address), which the wave runs whenever any lane keeps;
#     OPS_ARC per kept pair: its LDS reads, harmonic coefficients and the
#       never / always tests, the polynomial acos / atan2 of the clash arc and
#       its step range (marking the bitmask, 17 per 32-step word, is not
#       counted);
#     OPS_EVAL per (moving atom, non-bumping angle) evaluation: 6 FMA
#       rotation, 3 clamps, 3 conversions, 2 24-bit multiply-adds, shift and
#       the score add (the gather itself is a memory instruction).
OPS_PAIR, OPS_ROT, OPS_VOX = 8, 23, 22
OPS_CAND, OPS_ARC, OPS_EVAL = 13, 86, 16
# Rigid alignment, per (item, rotation, atom): 9 FMA rotation, 3 clamps,
# 3 conversions, shift, 2 24-bit multiply-adds and the score add (the gather
# is a memory instruction).
OPS_ALIGN = 19
ALIGN_ROTATIONS = 64

# Sources of the sweep kernel: the HBM traffic measured by the FETCH_SIZE /
# WRITE_SIZE counters is reported only while these are unchanged.
KERNEL_SOURCES = ("sweep_pruned.hip", "sweep_group.hip", "rotamer_step.h", "sweep_common.h",
                  "dock_internal.h")
TRAFFIC_FILES = {cfg: os.path.join(ROOT, "profiles", f"sweep_c{cfg}_traffic.md") for cfg in (2, 3, 5)}

WORKLOADS = {
    1: "C1: 64^3 pocket @0.5A, 1 ligand (32 atoms, 4 rotamers), 8 orientations, 64 steps",
    2: "C2: 128^3 pocket @0.375A, 10000 ligands (20-80 atoms, 2-12 rotamers), "
       "256 orientations, 256 steps",
    3: "C3: 128^3 pocket @0.375A, 100000 ligands (lognormal 8-150 atoms, 0-40 rotamers), "
       "128 orientations, 128 steps",
    5: "C5: 256^3 irregular pocket @0.25A, 2000 ligands (100-250 atoms, 60-120 rotamers), "
       "64 orientations, 360 steps",
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def batch_counts(ligs):
    """Per-batch sums over rotamers of m_r q_r and m_r (one orientation)."""
    n = np.diff(ligs.atom_offset).astype(np.int64)
    R = np.diff(ligs.rot_offset)
    lig_of_rot = np.repeat(np.arange(ligs.n_ligands), R)
    m = np.diff(ligs.move_offset).astype(np.int64)
    q = n[lig_of_rot] - m - 2
    return float((m * q).sum()), float(m.sum())


def dense_ops(ligs, n_orient, S):
    """Lane-operations of the unpruned sweep: every cross pair and every
    moving atom at every angle (the direct kernel's work)."""
    mq, msum = batch_counts(ligs)
    return (OPS_PAIR * mq + (OPS_ROT + OPS_VOX) * msum) * S * n_orient


def algorithmic_ops(ligs, n_orient, S, bump, kept_pairs, evals):
    """Lane-operations of one whole batch (see the unit costs above); the
    pruned kernel's kept pairs and evaluations are its own counts."""
    if bump == "direct":
        return dense_ops(ligs, n_orient, S)
    mq, _ = batch_counts(ligs)
    return OPS_CAND * mq * n_orient + OPS_ARC * kept_pairs + OPS_EVAL * evals


def kernel_sources_digest() -> str:
    """SHA-256 of the sweep kernel's code: the sources with comments removed
    and whitespace collapsed, so editing a comment keeps the digest."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1901_06229_amd", "csrc", name)) as f:
            code = f.read()
        code = re.sub(r"/\*.*?\*/", " ", code, flags=re.S)
        code = re.sub(r"//[^\n]*", " ", code)
        h.update(" ".join(code.split()).encode())
    return h.hexdigest()


def measured_traffic(cfg):
    """HBM bytes per sweep launch of this workload from the committed counter
    summary, if it was taken on the current kernel sources (else None)."""
    path = TRAFFIC_FILES.get(cfg)
    if path is None:
        return None
    try:
        with open(path) as f:
            fields = dict(l.split(":", 1) for l in f.read().splitlines() if l.startswith(("traffic_", "sources_")))
    except OSError:
        return None
    if fields.get("sources_sha256", "").strip() != kernel_sources_digest():
        return None
    return float(fields["traffic_bytes_per_launch"])


def gather_probe(grid_floats, blocks=4096, iters=256):
    """Random 4-byte gather rate of the part (the library's probe kernel): over
    2 MiB, which one XCD's L2 holds, and over a buffer of the grid's size."""
    import torch
    from paper_1901_06229_amd import dock
    out = torch.empty(blocks * 256, device="cuda:0")
    res = {}
    for name, log2 in (("2MiB", 19), ("grid_size", max(6, int(np.ceil(np.log2(grid_floats)))))):
        buf = torch.ones(1 << log2, device="cuda:0")
        dock.dock_probe_gather(buf, out, log2, blocks, iters)
        ms = min(dock.dock_probe_gather(buf, out, log2, blocks, iters) for _ in range(3))
        res[name] = {"bytes": 4 << log2, "gathers_per_s": round(blocks * 256 * iters / (ms / 1e3), 1)}
    return res


def valu_probe(blocks=8192, iters=4096):
    """Sustained VALU issue rate of the part (the library's probe kernel):
    FP32 FMA chains, and the sweep's per-evaluation instruction mix, in
    lane-ops per second; best of three runs each."""
    import torch
    from paper_1901_06229_amd import dock
    out = torch.empty(blocks * 256, device="cuda:0")
    res = {}
    for name, kind, ops in (("fma", 0, 1), ("eval_mix", 1, 16)):
        dock.dock_probe_valu(out, kind, blocks, iters)
        ms = min(dock.dock_probe_valu(out, kind, blocks, iters) for _ in range(3))
        res[name] = round(blocks * 256 * 8 * iters * ops / (ms / 1e3) / 1e12, 2)
    res["unit"] = "T lane-ops/s"
    res["note"] = ("issue-rate ceilings measured on this part: independent FP32 FMA chains, and the "
                   "sweep's 16-instruction evaluation (6 FMA, 3 clamps, 3 conversions, 2 24-bit "
                   "multiply-adds, conversion, add); packed FP32 is not used")
    return res


def copy_calibration():
    """A plain 1 GiB device-to-device copy, three times: the reference the
    FETCH_SIZE / WRITE_SIZE counters are scaled by."""
    import torch
    n = 1 << 28
    src = torch.ones(n, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print("copied 1 GiB x 3", flush=True)


def device_batch(ligs, orient, want_all=False):
    """CSR batch, orientations and result buffers as device tensors."""
    import torch
    from paper_1901_06229_amd import dock
    dev = torch.device("cuda:0")
    d = dict(n_ligands=ligs.n_ligands, total_atoms=int(ligs.atom_offset[-1]),
             total_rot=int(ligs.rot_offset[-1]), total_move=int(ligs.move_offset[-1]))
    for k, dt in (("atom_offset", torch.int32), ("xyz", torch.float32), ("rot_offset", torch.int32),
                  ("rot_axis", torch.int32), ("move_offset", torch.int32), ("move_atoms", torch.int16)):
        d[k] = torch.from_numpy(np.ascontiguousarray(getattr(ligs, k))).to(dev, dt)
    L, NA, NR = ligs.n_ligands, d["total_atoms"], d["total_rot"]
    out = dict(best_score=torch.empty(L, device=dev),
               best_orient=torch.empty(L, dtype=torch.int32, device=dev),
               angle_idx=torch.empty(max(NR, 1), dtype=torch.int16, device=dev),
               xyz=torch.empty(max(NA, 1), 3, device=dev),
               status=torch.empty(L, dtype=torch.int32, device=dev),
               n_fallback=torch.empty(L, dtype=torch.int32, device=dev))
    return d, torch.from_numpy(np.ascontiguousarray(orient)).to(dev), out


def time_steps(h, d, od, S, out, prm, ws, stream, steps, warmup):
    """Wall time per dock_batch_async step (inputs resident), synchronised."""
    import torch
    from paper_1901_06229_amd import dock
    for _ in range(warmup):
        dock.dock_batch_async(h, d, od, S, out, prm, workspace=ws, stream=stream)
    stream.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        dock.dock_batch_async(h, d, od, S, out, prm, workspace=ws, stream=stream)
    stream.synchronize()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def learned_comparison(n_eval=10_000, n_val=2_000, n_train=156_250, epochs=10, top_k=16,
                       steps=5, proposal=None, fine_steps=4096):
    """Plain vs learned proposal on the learned-proposal workload (64^3 pocket,
    32-atom 4-rotamer ligands, 8 orientations), same inputs, at S = 256 (one
    step per prediction bin) and at S = fine_steps (fine_steps / 256 steps per
    bin; same network)."""
    import torch
    from paper_1901_06229_amd import dock, learned, synth
    t0 = time.perf_counter()
    if proposal:
        net = dock.Mlp(learned.load_params(proposal))
        hist = {"loaded": proposal}
    else:
        net, hist = learned.train(n_ligands=n_train, epochs=epochs, log=log)
    t_train = time.perf_counter() - t0
    pocket = synth.pocket(learned.LEARN_CONFIG)
    h = dock.dock_init_pocket(pocket.grid, pocket.origin, pocket.spacing)
    dock.dock_load_proposal(h, net)
    orient = synth.orientations(learned.LEARN_CONFIG)
    stream = torch.cuda.Stream()
    batches = {}
    for name, first, count in (("val", n_eval, n_val), ("eval", 0, n_eval)):
        ligs = synth.ligands(learned.LIGAND_RECIPE, count=count, first=first,
                             seed=synth.config_seed(learned.LEARN_CONFIG), stream=synth.STREAM_EVAL)
        batches[name] = (ligs,) + device_batch(ligs, orient)

    def loss(sp, sl):
        return float(np.mean((sp - sl) / np.maximum(np.abs(sp), 1.0)))

    def compare(S):
        ws = {name: torch.empty(dock.dock_workspace_size(b[0].n_ligands, b[1]["total_rot"], 8, S),
                                dtype=torch.uint8, device="cuda") for name, b in batches.items()}

        def run(name, mode, margin, n_steps):
            ligs, d, od, out = batches[name]
            prm = dock.make_params(mode=mode, top_k=top_k, margin=margin, max_atoms=32, max_rot=4)
            sec = time_steps(h, d, od, S, out, prm, ws[name], stream, n_steps, 1)
            return sec, out["best_score"].cpu().numpy().copy(), int(out["n_fallback"].sum().item())

        # threshold on the validation ligands: fastest margin with <= 0.5 % mean loss
        _, sp_val, _ = run("val", dock.DOCK_MODE_PLAIN, 0.0, 1)
        candidates = []
        for tau in (-1.0, 0.02, 0.05, 0.1, 0.2, 0.4, 0.8, 3.0e38):
            sec, sl, nfb = run("val", dock.DOCK_MODE_LEARNED, tau, 2)
            candidates.append((tau, sec, loss(sp_val, sl), nfb / (n_val * 8 * 4)))
            log(f"S {S} val tau {tau:g}: {sec * 1e3:.3f} ms, loss {candidates[-1][2]:.5f}, "
                f"fallback {candidates[-1][3]:.3f}")
        ok = [c for c in candidates if c[2] <= 0.005]
        tau = min(ok, key=lambda c: c[1])[0] if ok else 3.0e38
        sec_p, sp, _ = run("eval", dock.DOCK_MODE_PLAIN, 0.0, steps)
        sec_l, sl, nfb = run("eval", dock.DOCK_MODE_LEARNED, tau, steps)
        net0 = dock.Mlp(learned.init_params(12345))
        dock.dock_load_proposal(h, net0)
        _, sl0, _ = run("eval", dock.DOCK_MODE_LEARNED, -1.0, 1)
        dock.dock_load_proposal(h, dock.Mlp(learned.stride_params(top_k)))
        _, sl_s, _ = run("eval", dock.DOCK_MODE_LEARNED, -1.0, 1)
        dock.dock_load_proposal(h, net)
        _, sl_t, _ = run("eval", dock.DOCK_MODE_LEARNED, -1.0, 1)
        return {
            "workload": f"learned proposal: 64^3 pocket @0.5A, {n_eval} held-out ligands (32 atoms, "
                        f"4 rotamers), 8 orientations, {S} steps ({S // 256} per prediction bin)",
            "angle_steps": S,
            "plain_ligands_per_s": round(n_eval / sec_p, 1),
            "learned_ligands_per_s": round(n_eval / sec_l, 1),
            "speedup": round(sec_p / sec_l, 3),
            "top_k": top_k, "margin_tau": tau if tau < 1e30 else "inf (full fallback)",
            "score_loss_mean": loss(sp, sl), "fallback_rate": nfb / (n_eval * 8 * 4),
            "no_fallback_loss_trained": loss(sp, sl_t), "no_fallback_loss_untrained": loss(sp, sl0),
            f"no_fallback_loss_stride{top_k}": loss(sp, sl_s),
            "validation": [{"tau": c[0] if c[0] < 1e30 else "inf", "ms": round(c[1] * 1e3, 3),
                            "loss": round(c[2], 5), "fallback": round(c[3], 3)} for c in candidates],
        }

    res = compare(256)
    if fine_steps:
        res["fine_steps"] = compare(fine_steps)
    fallback = {256: res["fallback_rate"]}
    if fine_steps:
        fallback[fine_steps] = res["fine_steps"]["fallback_rate"]
    res["bound"] = learned_bound(h, batches["eval"], n_eval, net, stream, fallback)
    h.close()
    res["training"] = {k: v for k, v in hist.items() if k not in ("train_loss", "val_loss")} | {
        "final_val_mse": hist.get("val_loss", [None])[-1], "seconds": round(t_train, 2)}
    return res, net


def learned_bound(h, batch, n_eval, net, stream, fallback, proposals=16, reps=10):
    """Speed bound on any learned proposal for the evaluation batch: the plain
    sweep at each step count S and at `proposals` steps (a rotamer step that
    tests and scores only that many angles), and the MLP over every item once
    per rotamer step, measured and at the MFMA peak.  Without fallback a
    learned call costs at least MLP + sweep(proposals); with a fallback rate
    f (the one the comparison measured at S) at least MLP + f sweep(S) +
    (1 - f) sweep(proposals)."""
    import torch
    from paper_1901_06229_amd import dock
    ligs, d, od, out = batch
    n_rot = int(np.diff(ligs.rot_offset).max())
    rows = n_eval * od.shape[0]

    def sweep_ms(S):
        ws = torch.empty(dock.dock_workspace_size(ligs.n_ligands, d["total_rot"], 8, S),
                         dtype=torch.uint8, device="cuda")
        prm = dock.make_params(max_atoms=32, max_rot=4, flags=dock.DOCK_FLAG_TIME_SWEEP)
        ms = []
        for i in range(reps + 2):
            dock.dock_batch_async(h, d, od, S, out, prm, workspace=ws, stream=stream)
            stream.synchronize()
            if i >= 2:
                ms.append(dock.dock_last_sweep_ms(h))
        return float(np.median(ms))

    x = torch.zeros(rows, 64, dtype=torch.bfloat16, device="cuda")
    y = torch.empty(rows, 256, dtype=torch.float32, device="cuda")
    for _ in range(3):
        net.forward(x, y, stream=stream)
    stream.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        net.forward(x, y, stream=stream)
    stream.synchronize()
    mlp_ms = (time.perf_counter() - t0) / reps * 1e3 * n_rot
    mlp_flop = 2.0 * rows * n_rot * (64 * 256 + 3 * 256 * 256)
    mlp_peak_ms = mlp_flop / MFMA_BF16_PEAK * 1e3
    small = sweep_ms(proposals)
    res = {"note": f"sweep ms (HIP events, median of {reps}) on the evaluation batch; a learned call needs "
                   f"the MLP on every item at each of {n_rot} rotamer steps plus at least a rotamer step "
                   f"that tests and scores {proposals} angles",
           f"plain_sweep_ms_{proposals}_steps": round(small, 4),
           "mlp_ms_measured": round(mlp_ms, 4), "mlp_ms_at_peak": round(mlp_peak_ms, 4)}
    for S, f in fallback.items():
        full = sweep_ms(S)
        with_fb = f * full + (1.0 - f) * small
        res[f"S{S}"] = {"plain_sweep_ms": round(full, 4),
                        "bound_no_fallback_measured_mlp": round(full / (small + mlp_ms), 3),
                        "bound_no_fallback_peak_mlp": round(full / (small + mlp_peak_ms), 3),
                        "fallback_rate": round(f, 3),
                        "bound_at_fallback_measured_mlp": round(full / (with_fb + mlp_ms), 3),
                        "bound_at_fallback_peak_mlp": round(full / (with_fb + mlp_peak_ms), 3),
                        "break_even_fallback_measured_mlp": round(
                            max(0.0, (full - small - mlp_ms) / (full - small)) if full > small else 0.0, 3)}
    return res


def learned_side_by_side(h, ligs, orient, d, orient_d, S, out, stream, steps, warmup, max_atoms,
                         net, plain_best, plain_step_s, n_val=200, top_k=16):
    """Plain and learned sweep side by side on this batch (the large-ligand
    workload), the proposal being the network trained on the learned-proposal
    workload's profiles.  The margin is the smallest of a grid that keeps the
    mean best-score loss against the plain sweep within 0.5 % on the first
    n_val ligands; then the whole batch is timed in learned mode."""
    import torch
    from paper_1901_06229_amd import dock, synth
    dock.dock_load_proposal(h, net)
    L = ligs.n_ligands
    max_rot = int(np.diff(ligs.rot_offset).max())

    def loss(sp, sl):
        return float(np.mean((sp - sl) / np.maximum(np.abs(sp), 1.0)))

    val = ligs.subset(range(min(n_val, L)))
    val_plain = dock.dock_batch(h, val, orient, S, r_bump=synth.R_BUMP)["best_score"]
    tried, tau = [], 3.0e38
    for t in (-1.0, 0.02, 0.05, 0.1, 0.2, 0.4, 0.8):
        r = dock.dock_batch(h, val, orient, S, r_bump=synth.R_BUMP, mode=dock.DOCK_MODE_LEARNED,
                            top_k=top_k, margin=t)
        tried.append({"tau": t, "loss": round(loss(val_plain, r["best_score"]), 5),
                      "fallback": round(float(r["n_fallback"].sum())
                                        / (orient.shape[0] * max(1, int(val.rot_offset[-1]))), 3)})
        log(f"side by side: val tau {t:g}: loss {tried[-1]['loss']:.5f}")
        if tried[-1]["loss"] <= 0.005:
            tau = t
            break
    ws = torch.empty(dock.dock_workspace_size(L, d["total_rot"], orient.shape[0], S), dtype=torch.uint8,
                     device="cuda:0")
    prm = dock.make_params(r_bump=synth.R_BUMP, mode=dock.DOCK_MODE_LEARNED, top_k=top_k, margin=tau,
                           max_atoms=max_atoms, max_rot=max_rot)
    out = dict(out, n_fallback=torch.zeros(L, dtype=torch.int32, device="cuda:0"))
    sec = time_steps(h, d, orient_d, S, out, prm, ws, stream, steps, warmup)
    learned_best = out["best_score"].cpu().numpy().copy()
    n_fb = int(out["n_fallback"].sum().item())
    return {
        "angle_steps": S, "top_k": top_k, "margin_tau": tau if tau < 1e30 else "inf (full fallback)",
        "plain_ligands_per_s": round(L / plain_step_s, 1),
        "learned_ligands_per_s": round(L / sec, 1),
        "speedup": round(plain_step_s / sec, 3),
        "score_loss_mean": loss(plain_best, learned_best),
        "score_loss_median": float(np.median((plain_best - learned_best) / np.maximum(np.abs(plain_best), 1.0))),
        "ligands_losing_over_0.5pct": float(np.mean((plain_best - learned_best)
                                                    / np.maximum(np.abs(plain_best), 1.0) > 0.005)),
        "fallback_rate": n_fb / float(orient.shape[0] * int(ligs.rot_offset[-1])),
        "validation": tried,
    }, learned_best


def align_leg(cfg, h, ligs, d, orient_d, S, out, stream, steps, warmup, max_atoms, n_align):
    """The same batch with a rigid alignment search before the sweep (paper
    §3.1, first phase): n_align rotations per (ligand, orientation) restart."""
    import torch
    from paper_1901_06229_amd import dock, synth
    L, O = ligs.n_ligands, orient_d.shape[0]
    rots = torch.from_numpy(synth.align_rotations(cfg, n_align)).cuda()
    ws = torch.empty(dock.dock_workspace_size(L, d["total_rot"], O, S, n_align=n_align),
                     dtype=torch.uint8, device="cuda:0")
    prm = dock.make_params(r_bump=synth.R_BUMP, max_atoms=max_atoms, flags=dock.DOCK_FLAG_TIME_SWEEP,
                           align=rots)

    def step():
        dock.dock_batch_async(h, d, orient_d, S, out, prm, workspace=ws, stream=stream)
        return dock.dock_last_align_ms(h), dock.dock_last_sweep_ms(h)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    times = []
    t0 = time.perf_counter()
    for _ in range(steps):
        times.append(step())
    stream.synchronize()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    align_s = float(np.mean([t[0] for t in times])) / 1e3
    evals = float(n_align) * O * float(ligs.atom_offset[-1])
    achieved = OPS_ALIGN * evals / align_s / 1e12
    return {
        "workload": f"{WORKLOADS[cfg].split(':')[0]} batch with a rigid alignment search of {n_align} "
                    "rotations (identity first) per restart before the sweep",
        "n_align": n_align,
        "ligands_per_s": round(steps * L / elapsed, 2),
        "ms_per_step": round(1e3 * elapsed / steps, 3),
        "sweep_ms": round(float(np.mean([t[1] for t in times])), 3),
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TOPS, 2),
                     "unit": "TOP/s", "frac": round(achieved / VALU_PEAK_TOPS, 4), "traffic": None,
                     "kernel": "align_kernel", "kernel_ms": round(1e3 * align_s, 3),
                     "work": f"lane-ops: {OPS_ALIGN} per (restart, rotation, atom) rotate-and-score",
                     "rotation_atom_evals": int(evals),
                     "gathers_per_s": round(evals / align_s, 1)},
    }


def cpu_info() -> dict:
    """Host description for the oracle timings: model, logical CPUs and the
    CPUs this process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for l in f:
                if l.startswith("model name"):
                    model = l.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except AttributeError:
        allowed = os.cpu_count()
    return {"model": model, "nproc": os.cpu_count(), "allowed": allowed}


def upload(ligs, orient, n_orient, S, want_all=False):
    """CSR batch, orientation table, results and workspace as device tensors."""
    import torch
    from paper_1901_06229_amd import dock
    dev = torch.device("cuda:0")
    d = dict(n_ligands=ligs.n_ligands, total_atoms=int(ligs.atom_offset[-1]),
             total_rot=int(ligs.rot_offset[-1]), total_move=int(ligs.move_offset[-1]))
    for k, dt in (("atom_offset", torch.int32), ("xyz", torch.float32), ("rot_offset", torch.int32),
                  ("rot_axis", torch.int32), ("move_offset", torch.int32), ("move_atoms", torch.int16)):
        d[k] = torch.from_numpy(np.ascontiguousarray(getattr(ligs, k))).to(dev, dt)
    L, NA, NR = ligs.n_ligands, d["total_atoms"], d["total_rot"]
    out = dict(best_score=torch.empty(L, device=dev), best_orient=torch.empty(L, dtype=torch.int32, device=dev),
               angle_idx=torch.empty(max(NR, 1), dtype=torch.int16, device=dev),
               xyz=torch.empty(max(NA, 1), 3, device=dev),
               status=torch.empty(L, dtype=torch.int32, device=dev))
    ws = torch.empty(dock.dock_workspace_size(L, NR, n_orient, S), dtype=torch.uint8, device=dev)
    return d, torch.from_numpy(np.ascontiguousarray(orient)).to(dev), out, ws


def plain_leg(cfg, steps, warmup, bump="pruned", waves=0, claim=16, autotune=0, graph=False,
              n_ligands=0, end_to_end=True):
    """Time the plain batched sweep on one workload: warm-up steps, then
    `steps` dock_batch_async calls enqueued back to back on resident inputs.
    Returns (result dict, context for the legs that reuse the batch)."""
    import torch
    from paper_1901_06229_amd import dock, synth
    preset = synth.PRESETS[cfg]
    S, O = preset["angle_steps"], preset["n_orient"]
    L = n_ligands or preset["n_ligands"]
    log(f"config {cfg}: generating {L} ligands")
    pocket = synth.pocket(cfg)
    ligs = synth.ligands(cfg, count=L)
    orient = synth.orientations(cfg)
    h = dock.dock_init_pocket(pocket.grid, pocket.origin, pocket.spacing)
    d, orient_d, out, ws = upload(ligs, orient, O, S)
    max_atoms = int(np.diff(ligs.atom_offset).max())
    flags = dock.DOCK_FLAG_TIME_SWEEP | (dock.DOCK_FLAG_DIRECT_BUMP if bump == "direct" else 0)
    if graph:
        flags |= dock.DOCK_FLAG_GRAPH
    prm = dock.make_params(r_bump=synth.R_BUMP, max_atoms=max_atoms, flags=flags)
    dock.dock_set_launch(h, waves, 0, claim)
    tune = None
    if autotune > 0:
        log(f"config {cfg}: autotuning the launch mapping on {autotune} sampled ligands")
        tune = dock.dock_autotune(h, ligs, orient, S, sample_ligands=min(autotune, L), seed=1,
                                  r_bump=synth.R_BUMP, flags=flags & dock.DOCK_FLAG_DIRECT_BUMP)
    launch = dict(zip(("waves_per_block", "blocks_per_cu", "items_per_claim"), dock.dock_get_launch(h)))
    launch.update(zip(("group16_atoms", "group32_atoms"), dock.dock_get_group_mapping(h)))
    launch["group32_split"] = dock.dock_get_group_split(h)
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()

    def step():
        dock.dock_batch_async(h, d, orient_d, S, out, prm, workspace=ws, stream=stream)

    for w in range(warmup):
        step()
        log(f"config {cfg}: warmup {w}: sweep {dock.dock_last_sweep_ms(h):.1f} ms")
    torch.cuda.synchronize()
    # the timed steps are enqueued back to back (no host wait between them);
    # the library keeps the sweep events of the last 16 timed calls, read
    # after the loop, in chunks of up to 16 steps
    sweep_ms = []
    t0 = time.perf_counter()
    for s in range(steps):
        step()
        if (s + 1) % 16 == 0 or s + 1 == steps:
            sweep_ms += dock.dock_sweep_ms_history(h, s + 1 - len(sweep_ms))
    stream.synchronize()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kept_pairs, evals = dock.dock_last_sweep_work(h)  # the same batch every step: the same counters
    # checked after the timed steps: a torch kernel between the warm-up and the
    # first timed sweep made that sweep ~1.3 ms slower on the 256 x 256 batch
    assert int((out["status"] != 0).sum()) == 0
    log(f"config {cfg}: sweep ms per step " + " ".join(f"{ms:.2f}" for ms in sweep_ms))
    value = steps * L / elapsed
    best = out["best_score"].cpu().numpy().copy()
    ops = algorithmic_ops(ligs, O, S, bump, kept_pairs, evals)
    mean_s = float(np.mean(sweep_ms)) / 1e3
    achieved = ops / mean_s / 1e12
    mq, msum = batch_counts(ligs)
    probe = gather_probe(int(np.prod(pocket.grid.shape)))
    res = {
        "value": round(value, 2), "unit": "ligands/s", "steps": steps, "warmup": warmup,
        "ms_per_step": round(1e3 * elapsed / steps, 3),
        "launch": dict(launch, autotuned=tune is not None, graph=graph,
                       **({"tune_entries": len(tune)} if tune else {})),
        "config": {"workload": WORKLOADS[cfg] if L == preset["n_ligands"] else
                   WORKLOADS[cfg] + f" (ligands overridden to {L})",
                   "n_ligands": L, "n_orient": O, "angle_steps": S, "r_bump": synth.R_BUMP},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TOPS, 2),
                     "unit": "TOP/s", "frac": round(achieved / VALU_PEAK_TOPS, 4),
                     "traffic": measured_traffic(cfg) if (bump == "pruned" and L == preset["n_ligands"])
                     else None,
                     "kernel": (("sweep_group_kernel<16>, sweep_group_kernel<32>, sweep_pruned_kernel "
                                 "(one launch per size class, timed together)")
                                if bump == "pruned" and any(launch[k] for k in ("group16_atoms", "group32_atoms"))
                                else "sweep_pruned_kernel" if bump == "pruned" else "sweep_kernel"),
                     "kernel_ms": round(1e3 * mean_s, 3),
                     **({"timed": "around each replayed graph (preparation, sweep, finalize)"}
                        if graph else {}),
                     "work": (f"lane-ops: {OPS_CAND} per candidate pair per rotamer step + "
                              f"{OPS_ARC} per kept pair (clash arc) + {OPS_EVAL} per (moving atom, "
                              "non-bumping angle) evaluation")
                     if bump == "pruned" else
                     "dense lane-ops per angle: 8 per cross pair + 45 per moving atom",
                     "candidate_pairs": int(mq * O), "kept_pairs": kept_pairs,
                     "atom_angle_evals": evals,
                     "valid_angle_frac": round(evals / (msum * O * S), 4) if msum else None,
                     "gathers": {
                         "per_s": round(evals / mean_s, 1),
                         "probe": probe,
                         "note": "voxel gathers of the scoring loop (one per evaluation) per second "
                                 "of the kernel, next to the probe's random 4-byte gathers; neighbouring "
                                 "angles share cache lines, so the kernel can exceed the probe"},
                     "dense_equivalent": {
                         "unit": "TOP/s",
                         "value": round(dense_ops(ligs, O, S) / mean_s / 1e12, 2),
                         "note": "lane-ops the unpruned sweep would execute (every pair and "
                                 "atom at every angle) per second of this kernel; not a "
                                 "fraction of peak"}},
    }
    if end_to_end:
        # the synchronous host-array call: H2D of the batch, the kernels, D2H
        # of the results (pageable numpy arrays); 1 warm-up, median of 5
        times = []
        for rep in range(6):
            t0 = time.perf_counter()
            r = dock.dock_batch(h, ligs, orient, S, r_bump=synth.R_BUMP)
            if rep:
                times.append(time.perf_counter() - t0)
        assert np.array_equal(r["best_score"], best), "synchronous and resident runs disagree"
        med = float(np.median(times))
        res["end_to_end"] = {
            "call": "dock_batch on host arrays: H2D + kernels + D2H, pageable host memory",
            "runs": [round(1e3 * t, 3) for t in times], "median_ms": round(1e3 * med, 3),
            "ligands_per_s": round(L / med, 2)}
        log(f"config {cfg}: end to end {1e3 * med:.2f} ms ({L / med:,.0f} ligands/s)")
    ctx = dict(h=h, pocket=pocket, ligs=ligs, orient=orient, d=d, orient_d=orient_d, out=out,
               stream=stream, S=S, O=O, max_atoms=max_atoms, best=best, step_s=elapsed / steps,
               workload=res["config"]["workload"])
    return res, ctx


def oracle_check(ctx, gpu_best, budget_s=16.0):
    """Per-ligand best-score error of GPU runs against the FP64 reference on
    the first ligands of the batch (as many as fit the time budget)."""
    import oracle
    from paper_1901_06229_amd import synth
    threads = min(16, cpu_info()["allowed"] or 1)
    ligs = ctx["ligs"]
    # one ligand per thread at the least (the reference runs one thread per ligand)
    n, ref, t_used = min(threads, ligs.n_ligands), None, 0.0
    while True:
        sub = ligs.subset(range(n))
        t0 = time.perf_counter()
        ref = oracle.dock_batch(ctx["pocket"], sub, ctx["orient"], ctx["S"], r_bump=synth.R_BUMP,
                                n_threads=threads).best_score
        t_used = time.perf_counter() - t0
        if t_used >= budget_s / 2 or n * 2 > ligs.n_ligands:
            break
        n *= 2
    out = {"ligands": n, "seconds": round(t_used, 1)}
    for name, b in gpu_best.items():
        err = (ref - b[:n]) / np.maximum(np.abs(ref), 1.0)
        out[name] = {"max_abs_rel_err": float(np.max(np.abs(err))),
                     "mean_abs_rel_err": float(np.mean(np.abs(err))),
                     "mean_loss": float(np.mean(err)), "per_ligand_rel_err": [float(x) for x in err]}
    return out


def cpu_baseline(ctx, budget_s=16.0, single_s=6.0):
    """The FP64 reference on bounded samples of the headline workload (the
    first ligands, doubling the count until one run takes at least half the
    budget): on every CPU this process may use (at most 16, the host share
    of one GPU) and on one core."""
    import oracle
    from paper_1901_06229_amd import synth
    info = cpu_info()
    threads = max(1, min(16, info["allowed"] or 1))
    ligs = ctx["ligs"]

    def rate(n_threads, budget):
        n = max(1, n_threads)
        while True:
            sub = ligs.subset(range(n))
            t0 = time.perf_counter()
            oracle.dock_batch(ctx["pocket"], sub, ctx["orient"], ctx["S"], r_bump=synth.R_BUMP,
                              n_threads=n_threads)
            t = time.perf_counter() - t0
            if t >= budget / 2 or n * 2 > ligs.n_ligands:
                return n, t
            n *= 2

    n_all, t_all = rate(threads, budget_s)
    n_one, t_one = rate(1, single_s)
    return {"value": n_all / t_all, "unit": "ligands/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n_all} ligands of the headline workload, all orientations and steps, "
                      f"FP64, {threads} threads, {t_all:.1f} s",
            "single_core": {"value": n_one / t_one, "sample": f"first {n_one} ligands, 1 thread, {t_one:.1f} s"},
            "host": info}


def hybrid_leg(ctx, runs=3):
    """Node throughput with host threads beside the GPU (paper §4.2 and §5.1:
    CPU processes add to the GPU process): the same host-array batch docked
    by the GPU alone (pipelined chunks, no host threads) and by the GPU with
    host threads from the same dispenser; then the host threads alone on a
    bounded sample.  Median of `runs` after one warm-up each."""
    from paper_1901_06229_amd import dock, synth
    h, ligs, orient, S = ctx["h"], ctx["ligs"], ctx["orient"], ctx["S"]
    L = ligs.n_ligands
    threads = max(0, min(16, cpu_info()["allowed"] or 1) - 1)

    def timed(**kw):
        times, res = [], None
        for rep in range(runs + 1):
            t0 = time.perf_counter()
            res = dock.dock_batch_hybrid(h, ligs, orient, S, r_bump=synth.R_BUMP, **kw)
            if rep:
                times.append(time.perf_counter() - t0)
        return float(np.median(times)), res

    t_gpu, r_gpu = timed(cpu_threads=0)
    assert np.array_equal(r_gpu["best_score"], ctx["best"]), "hybrid GPU-only run disagrees"
    t_hyb, r_hyb = timed(cpu_threads=threads)
    gpu_l = r_hyb["done_by"] == 0
    assert np.array_equal(r_hyb["best_score"][gpu_l], ctx["best"][gpu_l])
    log(f"hybrid: GPU only {L / t_gpu:,.0f} ligands/s, GPU + {threads} host threads "
        f"{L / t_hyb:,.0f} ligands/s ({r_hyb['stats']['cpu_ligands']} ligands on the host)")
    # host threads alone on the first ligands (about 3 s)
    n = 64
    while True:
        sub = ligs.subset(range(n))
        t0 = time.perf_counter()
        dock.dock_batch_hybrid(h, sub, orient, S, r_bump=synth.R_BUMP, cpu_threads=threads, use_gpu=False)
        t_host = time.perf_counter() - t0
        if t_host >= 1.5 or 2 * n > L:
            break
        n *= 2
    return {
        "workload": ctx["workload"] + ", host arrays in and out",
        "gpu_only_ligands_per_s": round(L / t_gpu, 1),
        "hybrid_ligands_per_s": round(L / t_hyb, 1),
        "gain": round(t_gpu / t_hyb, 4),
        "host_threads": threads,
        "host_ligands": int(r_hyb["stats"]["cpu_ligands"]),
        "gpu_chunks": int(r_hyb["stats"]["gpu_chunks"]),
        "ms": {"gpu_only": round(1e3 * t_gpu, 2), "hybrid": round(1e3 * t_hyb, 2)},
        "host_only": {"ligands_per_s": round(n / t_host, 1), "threads": threads,
                      "sample": f"first {n} ligands, FP32 host sweep (AVX2), {t_host:.2f} s"},
        "note": "gpu_only is the same call with no host threads (GPU chunks pipelined with their "
                "copies); host-only rate of the product FP32 CPU sweep, not the FP64 reference",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    # the first sweep after a batch is staged runs ~10 % slower
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=3, choices=sorted(WORKLOADS),
                    help="headline workload (default: the 100,000-ligand uneven batch)")
    ap.add_argument("--ligands", type=int, default=0, help="override the headline ligand count")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--bump", choices=("pruned", "direct"), default="pruned",
                    help="pruned: test only pairs that can clash; direct: every pair")
    ap.add_argument("--waves", type=int, default=0,
                    help="waves per block of the sweep (0: the most resident waves)")
    ap.add_argument("--claim", type=int, default=16,
                    help="most items a wave takes per work-queue atomic")
    ap.add_argument("--autotune", type=int, default=None,
                    help="time every launch mapping on this many sampled ligands first and keep "
                         "the fastest (default: the whole uneven batch, 100000 ligands; else off)")
    ap.add_argument("--graph", action=argparse.BooleanOptionalAction, default=None,
                    help="replay the batch's launch sequence as a captured HIP graph "
                         "(default: on for the uneven-batch workload)")
    ap.add_argument("--legs", default=None,
                    help="comma list of extra legs: hybrid (GPU and host threads on the headline "
                         "batch), c2 (the 10,000-ligand batch), c5 (large "
                         "ligands, plain and learned side by side), align, learned; default: all "
                         "for the uneven-batch headline, none otherwise")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-proposal legs")
    ap.add_argument("--align", type=int, default=ALIGN_ROTATIONS,
                    help="rotations of the rigid-alignment leg (0: skip it)")
    ap.add_argument("--no-end-to-end", action="store_true",
                    help="skip the synchronous host-array timing")
    ap.add_argument("--proposal", default=None, help="directory of trained proposal weights")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run the 1 GiB copy that calibrates the HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(a batch would shard by ligand, with no exchange between GPUs)", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration()
        return

    import torch
    torch.cuda.set_device(0)
    cfg = args.config
    legs = (args.legs.split(",") if args.legs is not None else
            (["hybrid", "c2", "c5", "align", "learned"] if cfg == 3 else []))
    legs = [x for x in legs if x]
    if args.no_learned:
        legs = [x for x in legs if x != "learned"]
    if args.align <= 0:
        legs = [x for x in legs if x != "align"]
    autotune = args.autotune if args.autotune is not None else (100000 if cfg == 3 else 0)
    graph = args.graph if args.graph is not None else cfg == 3
    head, ctx = plain_leg(cfg, args.steps, args.warmup, args.bump, args.waves, args.claim, autotune,
                          graph, args.ligands, end_to_end=not args.no_end_to_end)
    line = {
        "metric": METRIC, "value": head["value"], "unit": "ligands/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic", "mode": "plain", "bump": args.bump, "launch": head["launch"],
        "config": head["config"], "roofline": head["roofline"],
    }
    if "end_to_end" in head:
        line["end_to_end"] = head["end_to_end"]
    line["roofline"]["valu_probe"] = probe = valu_probe()
    line["roofline"]["frac_of_probe_fma"] = round(line["roofline"]["achieved"] / probe["fma"], 4)
    line["paper_context"] = {
        "note": "the paper (arXiv 1901.06229) prints no throughput for this path and no workload "
                "sizes (1500 unpublished ligands); its figures are context, not comparable",
        "optimize_pose_gpu_speedup": "2x, OpenACC on 1 Tesla K80 GK210 vs 2x 8-core Xeon E5-2630 v3 (§4.1)",
        "alignment_gpu_speedup": "16x, same hardware (§4.1)",
        "hybrid_node": "5.8 ligands/s, 16 OpenMP threads + 2 GK210 GPUs, whole docking incl. alignment (§5.2)",
    }
    if "hybrid" in legs:
        log("hybrid: GPU and host threads from one dispenser")
        line["hybrid"] = hybrid_leg(ctx)
    if not args.no_cpu_baseline:
        log("timing the FP64 reference on samples of the headline workload")
        line["cpu_baseline"] = cpu_baseline(ctx)
    net = None
    if "learned" in legs:
        log("learned proposal: training on the GPU and comparing with the plain sweep")
        line["learned"], net = learned_comparison(proposal=args.proposal)
    extra = {}
    for name, c in (("c2", 2), ("c5", 5)):
        if name not in legs or c == cfg:
            continue
        res, lctx = plain_leg(c, args.steps, args.warmup, args.bump, end_to_end=not args.no_end_to_end)
        gpu_best = {"plain": lctx["best"]}
        if c == 2 and "align" in legs:
            log(f"rigid alignment: {args.align} rotations per restart before the sweep")
            res["align"] = align_leg(c, lctx["h"], lctx["ligs"], lctx["d"], lctx["orient_d"], lctx["S"],
                                     lctx["out"], lctx["stream"], args.steps, args.warmup,
                                     lctx["max_atoms"], args.align)
        if c == 5 and net is not None:
            log("large-ligand workload: plain and learned sweep side by side")
            res["learned_side_by_side"], gpu_best["learned"] = learned_side_by_side(
                lctx["h"], lctx["ligs"], lctx["orient"], lctx["d"], lctx["orient_d"], lctx["S"],
                lctx["out"], lctx["stream"], args.steps, args.warmup, lctx["max_atoms"], net,
                lctx["best"], lctx["step_s"])
        if c == 5 and not args.no_cpu_baseline:
            log("large-ligand workload: per-ligand error against the FP64 reference")
            res["vs_oracle"] = oracle_check(lctx, gpu_best)
        lctx["h"].close()
        extra[name] = res
    line.update(extra)
    print(json.dumps(line), flush=True)
    ctx["h"].close()


if __name__ == "__main__":
    main()
