"""Training and evaluation driver of the learned angle proposal.

Python only orchestrates: profiles come from the GPU plain sweep
(``dock_emit_profiles``), the network is trained by the library's own BF16
MFMA forward/backward kernels and Adam (``Mlp.loss_grad`` / ``Mlp.adam``),
and inference runs inside ``dock_batch(mode=DOCK_MODE_LEARNED)``.  torch
provides device memory, random permutations of the training rows and
streams.

Workload (learned proposal): the 64^3 pocket, ligands from the 32-atom,
4-rotamer recipe, 8 orientations, 256 angle steps; training ligands from
generator stream 3, held-out evaluation ligands from stream 4.
"""
from __future__ import annotations

import json
import math
import os
import time

import numpy as np

from . import dock, synth

LEARN_CONFIG = 4        # recipe id of the learned-proposal workload
LIGAND_RECIPE = 1       # 32 atoms, 4 rotamers
S_BINS = 256


def init_params(seed: int = 0) -> np.ndarray:
    """Uniform(+-1/sqrt(fan_in)) weights, zero biases (packed FP32 layout)."""
    rng = np.random.default_rng(seed)
    parts = []
    for o, i in ((256, 64), (256, 256), (256, 256), (256, 256)):
        b = 1.0 / math.sqrt(i)
        parts.append(rng.uniform(-b, b, o * i))
        parts.append(np.zeros(o))
    return np.concatenate(parts).astype(np.float32)


def stride_params(k: int = 16) -> np.ndarray:
    """A network that ignores its input and predicts one fixed landscape: 1 on
    every (256 / k)-th bin, 0 elsewhere (all weights zero, GELU(0) = 0).  Its
    nominations are the non-learned stride proposal of the same top_k."""
    p = np.zeros_like(init_params(0))
    p[-S_BINS:][:: S_BINS // k] = 1.0
    return p


def emit_dataset(pocket_h, n_ligands: int, seed: int, stream: int, orient, chunk: int = 20000,
                 log=print):
    """Profiles of n_ligands training ligands as device tensors (x, t, mask)."""
    import torch
    xs, ts, ms = [], [], []
    done = 0
    while done < n_ligands:
        cnt = min(chunk, n_ligands - done)
        ligs = synth.ligands(LIGAND_RECIPE, count=cnt, first=done, seed=seed, stream=stream)
        rows = int(ligs.rot_offset[-1]) * orient.shape[0]
        x = torch.empty(rows, 64, dtype=torch.int16, device="cuda")
        t = torch.empty(rows, S_BINS, dtype=torch.int16, device="cuda")
        m = torch.empty(rows, 8, dtype=torch.int32, device="cuda")
        dock.dock_emit_profiles(pocket_h, ligs, orient, x, t, m)
        xs.append(x)
        ts.append(t)
        ms.append(m)
        done += cnt
        log(f"profiles: {done}/{n_ligands} ligands")
    return torch.cat(xs), torch.cat(ts), torch.cat(ms)


def train(n_ligands: int = 156_250, epochs: int = 10, batch: int = 4096, lr: float = 1e-3,
          seed: int = 0, val_frac: float = 0.01, log=print, out_dir: str | None = None):
    """Generate profiles on the GPU and train the proposal network there.

    Returns (Mlp, history dict)."""
    import torch
    torch.cuda.set_device(0)
    pocket = synth.pocket(LEARN_CONFIG)
    h = dock.dock_init_pocket(pocket.grid, pocket.origin, pocket.spacing)
    orient = synth.orientations(LEARN_CONFIG)
    t0 = time.perf_counter()
    X, T, _ = emit_dataset(h, n_ligands, synth.config_seed(LEARN_CONFIG), synth.STREAM_TRAIN, orient,
                           log=log)
    torch.cuda.synchronize()
    t_emit = time.perf_counter() - t0
    N = X.shape[0]
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    perm = torch.randperm(N, device="cuda", generator=g)
    n_val = max(batch, int(N * val_frac) // 64 * 64)
    val_idx, tr_idx = perm[:n_val], perm[n_val:]
    Xv, Tv = X[val_idx].contiguous(), T[val_idx].contiguous()
    net = dock.Mlp(init_params(seed))
    hist = {"profiles": int(N), "emit_s": t_emit, "train_loss": [], "val_loss": []}
    t1 = time.perf_counter()
    steps = 0
    for ep in range(epochs):
        order = tr_idx[torch.randperm(tr_idx.numel(), device="cuda", generator=g)]
        nb = order.numel() // batch
        ep_loss = 0.0
        for b in range(nb):
            rows = order[b * batch:(b + 1) * batch]
            xb, tb = X[rows].contiguous(), T[rows].contiguous()
            want = (b % 50 == 0) or b == nb - 1
            loss = net.loss_grad(xb, tb, want_loss=want)
            net.adam(lr=lr)
            steps += 1
            if want:
                ep_loss = loss
        vl = net.loss_grad(Xv, Tv, want_loss=True)
        hist["train_loss"].append(ep_loss)
        hist["val_loss"].append(vl)
        log(f"epoch {ep}: train {ep_loss:.4f} val {vl:.4f}")
    torch.cuda.synchronize()
    hist["train_s"] = time.perf_counter() - t1
    hist["steps"] = steps
    # forward 2 and backward 4 flops per multiply-accumulate
    hist["gflop"] = steps * batch * 6 * (64 * 256 + 3 * 256 * 256) / 1e9
    if out_dir:
        save_checkpoint(net, hist, out_dir)
    h.close()
    return net, hist


def save_checkpoint(net: "dock.Mlp", hist: dict, out_dir: str):
    os.makedirs(out_dir, exist_ok=True)
    np.save(os.path.join(out_dir, "proposal_params.npy"), net.get_params())
    with open(os.path.join(out_dir, "proposal_manifest.json"), "w") as f:
        json.dump({"layers": [[64, 256], [256, 256], [256, 256], [256, 256]],
                   "activation": "gelu(erf)", "dtype": "bf16 weights, fp32 master", **hist}, f)


def load_params(out_dir: str) -> np.ndarray:
    return np.load(os.path.join(out_dir, "proposal_params.npy"))
