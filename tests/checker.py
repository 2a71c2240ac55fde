"""Ambiguity-aware replay checker: GPU sweep vs the FP64 reference.

A voxel lookup and the bump threshold are step functions, so an FP32 pose can
land on the other side of a voxel face or of r_bump than the FP64 pose.  The
checker therefore replays the reference along the GPU's own angle choices and
accepts a different choice kg at a step only when
  * the reference finds kg valid, or kg has a cross pair within 1e-4 A of
    r_bump (the GPU may have found it valid), and
  * no angle the reference finds clearly valid beats kg: for each such k,
    kg's score plus 1e-5 max(|s|, 1) reaches k's score, where a score whose
    atoms sit within 1e-4 A of a voxel face counts as its interval of
    alternative-voxel sums (kg at its top, k at its bottom).
It is a 'tie' if the reference's own choice is clearly valid and within the
tolerance of kg's score, else 'ambiguous'; tests bound the ambiguous share.
Coordinates must then match within 1e-4 A and scores within 1e-5 relative
(or inside the reference's ambiguity interval, counted as score_band).
"""
from __future__ import annotations

from collections import Counter
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

import oracle

COORD_TOL = 1e-4
REL_TOL = 1e-5

V, VAMB, SAMB = oracle.FLAG_VALID, oracle.FLAG_VAMB, oracle.FLAG_SAMB


def tol_of(s: float) -> float:
    return REL_TOL * max(abs(s), 1.0)


@dataclass
class Report:
    steps: Counter = field(default_factory=Counter)
    failures: list = field(default_factory=list)
    items: int = 0
    score_band: int = 0     # final scores accepted only inside the reference's interval
    score_flagged: int = 0  # items whose reference final pose has an atom within the face band
    max_coord_err: float = 0.0
    max_score_rel: float = 0.0

    def ok(self) -> bool:
        return not self.failures

    def ambiguity_rates(self) -> tuple[float, float]:
        """(share of steps accepted through a flagged ambiguity, share of items
        whose final score is accepted only through its interval)."""
        n_steps = sum(v for k, v in self.steps.items() if not k.startswith("align_"))
        return (self.steps["ambiguous"] / max(1, n_steps), self.score_band / max(1, self.items))

    def assert_rare(self, step_frac: float = 0.01, flagged_frac: float = 0.5) -> None:
        """Acceptances through the ambiguity band must stay rare: at delta =
        1e-4 A an FP32 pose lands across a face or r_bump only occasionally.
        A final score can fall in its band only through an atom within delta
        of a voxel face (score_flagged counts those items); an FP32 pose off
        by ~1e-5 A crosses such a face in well under half of them, whereas a
        kernel that indexed voxels wrongly at faces would cross in nearly all.
        A batch of a few items may hold one or two such cases."""
        n_steps = sum(v for k, v in self.steps.items() if not k.startswith("align_"))
        amb_ok = max(2.0, step_frac * n_steps)
        band_ok = max(2.0, flagged_frac * self.score_flagged)
        assert self.steps["ambiguous"] <= amb_ok, f"too many ambiguous steps: {self.summary()}"
        assert self.score_band <= band_ok, f"too many band-accepted scores: {self.summary()}"

    def summary(self) -> str:
        return (f"items={self.items} steps={dict(self.steps)} score_band={self.score_band} "
                f"(of {self.score_flagged} flagged) "
                f"max|dx|={self.max_coord_err:.2e} "
                f"max score rel={self.max_score_rel:.2e} failures={len(self.failures)} "
                f"{self.failures[:5]}")


def classify_step(tr, s: int, kg: int) -> str | None:
    """'exact' / 'tie' / 'ambiguous', or None if the GPU choice is not acceptable.

    The GPU's angle kg must be one the GPU can have found valid (valid in the
    reference, or within the band of r_bump), and no angle the reference
    finds clearly valid may beat it: for every clearly valid k != kg,
    hi[kg] + tol >= lo[k] (lo = hi = s where no atom sits within the band of
    a voxel face).  It is a 'tie' when the reference's own choice is clearly
    valid and within tol of kg's plain score, otherwise 'ambiguous'."""
    ko = int(tr.k_star[s])
    if kg == ko:
        return "exact"
    f, sc, lo, hi = tr.prof_flags[s], tr.prof_s[s], tr.prof_lo[s], tr.prof_hi[s]
    clearly_valid = ((f & V) > 0) & ((f & VAMB) == 0)
    if kg == -1:
        return "ambiguous" if not clearly_valid.any() else None
    if kg < 0 or kg >= len(f):
        return None
    if not (f[kg] & (V | VAMB)):
        return None
    others = clearly_valid.copy()
    others[kg] = False
    tol = tol_of(sc[ko] if ko >= 0 else sc[kg])
    if others.any() and hi[kg] + tol < lo[others].max():
        return None
    if ko >= 0 and clearly_valid[ko] and clearly_valid[kg] and sc[ko] - sc[kg] <= tol:
        return "tie"
    return "ambiguous"


def classify_align(tr, ag: int) -> str | None:
    """The GPU's alignment choice against the reference's candidate scores."""
    ao = int(tr.a_star)
    if ag == ao:
        return "exact"
    if ag < 0 or ag >= len(tr.align_s):
        return None
    tol = tol_of(tr.align_s[ao])
    if tr.align_s[ao] - tr.align_s[ag] <= tol:
        return "tie"
    if tr.align_hi[ag] + tol >= tr.align_lo[ao]:
        return "ambiguous"
    return None


def check_item(pocket, lig, orient, S, r_bump, passes, gpu_k, gpu_score, gpu_xyz=None,
               align=None, gpu_a=-1):
    """Replay one item along the GPU's choices (its alignment first, if a
    rotation set is given); returns (counts, failures, dx, rel)."""
    tr = oracle.trace_item(pocket, lig, orient, S, r_bump, passes, forced_k=gpu_k, align=align,
                           forced_a=int(gpu_a) if align is not None else -1)
    counts, fails = Counter(), []
    if align is not None:
        c = classify_align(tr, int(gpu_a))
        if c is None:
            fails.append(("align", int(gpu_a), int(tr.a_star)))
        else:
            counts["align_" + c] += 1
    for s, kg in enumerate(gpu_k):
        c = classify_step(tr, s, int(kg))
        if c is None:
            fails.append(("step", s, int(kg), int(tr.k_star[s])))
        else:
            counts[c] += 1
    tol = tol_of(tr.score)
    rel = abs(gpu_score - tr.score) / max(abs(tr.score), 1.0)
    if tr.score_lo < tr.score_hi:
        counts["score_flagged"] += 1
    if abs(gpu_score - tr.score) > tol:
        if tr.score_lo - tol <= gpu_score <= tr.score_hi + tol:
            counts["score_band"] += 1
        else:
            fails.append(("score", float(gpu_score), tr.score, tr.score_lo, tr.score_hi))
    dx = 0.0
    if gpu_xyz is not None:
        dx = float(np.abs(np.asarray(gpu_xyz, np.float64) - tr.xyz).max()) if len(tr.xyz) else 0.0
        if dx > COORD_TOL:
            fails.append(("coords", dx))
    return counts, fails, dx, rel


def item_steps(ligs, l, o, O, passes, all_angle_idx):
    R = ligs.n_rot(l)
    base = (int(ligs.rot_offset[l]) * O + o * R) * passes
    return all_angle_idx[base:base + R * passes]


def check_batch(pocket, ligs, orient, S, res, r_bump=2.0, passes=1, ligands=None,
                orients=None, threads=8, align=None) -> Report:
    """Check GPU results ``res`` (dock_batch output with want_all=True).

    ligands: ligand indices to check (default all); orients: orientation
    indices per ligand (default all) -- the winning orientation is always
    checked, including its final coordinates.  align: the rotation set the
    GPU run aligned with (its choices are in res["all_align_idx"]).
    """
    O = orient.shape[0]
    rep = Report()
    ligands = range(ligs.n_ligands) if ligands is None else ligands
    jobs = []
    for l in ligands:
        l = int(l)
        lig = ligs.ligand(l)
        ob = int(res["best_orient"][l])
        if ob < 0:
            rep.failures.append(("rejected", l))
            continue
        osel = set(range(O) if orients is None else (int(x) for x in orients)) | {ob}
        for o in sorted(osel):
            k = item_steps(ligs, l, o, O, passes, res["all_angle_idx"])
            xyz = None
            if o == ob:
                a0, a1 = ligs.atom_offset[l], ligs.atom_offset[l + 1]
                xyz = res["xyz"][a0:a1]
            a = int(res["all_align_idx"][l, o]) if align is not None else -1
            jobs.append((l, o, lig, k, float(res["all_scores"][l, o]), xyz, a))

    def run(job):
        l, o, lig, k, sc, xyz, a = job
        return (l, o) + check_item(pocket, lig, orient[o], S, r_bump, passes, k, sc, xyz,
                                   align=align, gpu_a=a)

    with ThreadPoolExecutor(max(1, threads)) as ex:
        for l, o, counts, fails, dx, rel in ex.map(run, jobs):
            rep.items += 1
            rep.score_band += counts.pop("score_band", 0)
            rep.score_flagged += counts.pop("score_flagged", 0)
            rep.steps.update(counts)
            rep.max_coord_err = max(rep.max_coord_err, dx)
            rep.max_score_rel = max(rep.max_score_rel, rel)
            rep.failures.extend((l, o) + f for f in fails)
    # per-ligand reduction: GPU's own argmax over its scores, lowest index on ties
    for l in ligands:
        l = int(l)
        s = res["all_scores"][l]
        ob = int(res["best_orient"][l])
        if ob >= 0 and (ob != int(np.argmax(s)) or res["best_score"][l] != s[ob]):
            rep.failures.append(("best_orient", l, ob, int(np.argmax(s))))
        R = ligs.n_rot(l)
        if ob >= 0 and R:
            a = res["angle_idx"][int(ligs.rot_offset[l]) * passes:][:R * passes]
            if not np.array_equal(a, item_steps(ligs, l, ob, O, passes, res["all_angle_idx"])):
                rep.failures.append(("angle_idx", l))
        if align is not None and ob >= 0 and res["align_idx"][l] != res["all_align_idx"][l, ob]:
            rep.failures.append(("align_idx", l))
    return rep


def check_best_orientation(pocket, ligs, orient, S, res, ref, r_bump=2.0, ligands=None) -> list:
    """The GPU's winning orientation must be a reference winner up to ties or
    ambiguity: reference S(o*_gpu) within tolerance of the reference best."""
    bad = []
    ligands = range(ligs.n_ligands) if ligands is None else ligands
    for l in ligands:
        l = int(l)
        og, oo = int(res["best_orient"][l]), int(ref.best_orient[l])
        if og == oo:
            continue
        sg, so = ref.all_scores[l, og], ref.all_scores[l, oo]
        if so - sg <= tol_of(so):
            continue
        # the two items' GPU scores disagree with the reference ordering: only
        # acceptable if the GPU trajectory itself was ambiguity-accepted
        bad.append((l, og, oo, float(sg), float(so)))
    return bad
