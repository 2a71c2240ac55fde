"""The fixed-point pair bound keeps every pair the float bound keeps.

The sweep kernels store an atom's (z, |r|) about the bond axis as two int16
in units of 1/256 Angstrom (clamped to the int16 range, truncated toward
zero) and test a cross pair with a saturating packed subtract and a
saturating int16 dot product against a threshold widened by 3 units
(pack_zr, zr_bound, zr_threshold in the sweep's rotamer-step header).  The
cylinder bound itself is the paper's per-fragment validity test reduced to a
lower bound (section 4.1; the exact clash arcs decide afterwards).

This emulates those integer steps on the host and checks what the kernels
rely on: whenever the FP32 bound (dz^2 + dr^2) of the same coordinates is
below the float threshold r_bump^2 + margin, the quantised bound is at most
the integer threshold, so the kept pairs are a superset of the float test's
and every clash arc is marked as before.  It also checks the superset is
tight (pairs a few hundredths of an Angstrom beyond the threshold are
dropped), so a threshold that keeps everything would fail.
"""
import numpy as np

UNITS = 256.0
MARGIN = 1e-3  # the float test's margin on r_bump^2 (A^2)
I32_MAX = 2**31 - 1


def pack(z, r):
    zi = np.trunc(np.clip((np.float32(z) * np.float32(UNITS)).astype(np.float32), -32768, 32767))
    ri = np.trunc(np.minimum((np.float32(r) * np.float32(UNITS)).astype(np.float32), 32767))
    return zi.astype(np.int64), ri.astype(np.int64)


def quant_bound(a, b):
    dz = np.clip(a[0] - b[0], -32768, 32767)
    dr = np.clip(a[1] - b[1], -32768, 32767)
    return np.clip(dz * dz + dr * dr, -2**31, I32_MAX)


def threshold(thr):
    b = np.sqrt(np.float64(np.float32(thr))) * UNITS + 3.0
    return I32_MAX if b * b >= 2147483647.0 else int(b * b) + 1


def float_bound(zi, ri, zj, rj):
    dz = (zi - zj).astype(np.float32)
    dr = (ri - rj).astype(np.float32)
    dzz = (dz * dz).astype(np.float32)
    return (dr.astype(np.float64) * dr + dzz).astype(np.float32)  # fmaf(dr, dr, dz * dz)


def _pairs(rng, n, zscale, rscale, dist=None):
    zi = rng.uniform(-zscale, zscale, n).astype(np.float32)
    # with a target distance, radii start at it so r_j = r_i + d sin(phi)
    # stays non-negative and the pair keeps that distance
    lo = 0.0 if dist is None else np.max(dist)
    ri = rng.uniform(lo, rscale + lo, n).astype(np.float32)
    if dist is None:
        zj = rng.uniform(-zscale, zscale, n).astype(np.float32)
        rj = rng.uniform(0, rscale, n).astype(np.float32)
    else:  # partners at a given (z, r)-plane distance
        phi = rng.uniform(0, 2 * np.pi, n)
        zj = (zi + dist * np.cos(phi)).astype(np.float32)
        rj = (ri + dist * np.sin(phi)).astype(np.float32)
    return zi, ri, zj, rj


def test_quantised_bound_keeps_every_float_kept_pair():
    rng = np.random.default_rng(20260311)
    checked = 0
    for r_bump in (0.0, 0.4, 1.5, 2.8, 3.3, 12.0, 50.0, 140.0, 200.0):
        r2 = np.float32(r_bump) * np.float32(r_bump)
        thr = np.float32(r2 + np.float32(MARGIN))
        T = threshold(thr)
        for zscale, rscale in ((1.0, 1.0), (30.0, 20.0), (127.0, 127.0), (400.0, 300.0)):
            for dist in (None, np.sqrt(thr) * (1 - rng.uniform(0, 1e-3, 20000)),
                         np.sqrt(thr) * rng.uniform(0.0, 1.0, 20000)):
                zi, ri, zj, rj = _pairs(rng, 20000, zscale, rscale, dist)
                keep_f = float_bound(zi, ri, zj, rj) < thr
                qb = quant_bound(pack(zi, ri), pack(zj, rj))
                keep_q = qb <= T
                missed = keep_f & ~keep_q
                assert not missed.any(), (r_bump, zscale, int(missed.sum()))
                checked += int(keep_f.sum())
    assert checked > 200000  # most of the boundary samples are float-kept pairs


def test_quantised_bound_is_tight():
    """Away from saturation, pairs 0.03 A beyond the threshold distance are
    dropped: the widening is a few units, not a keep-everything threshold."""
    rng = np.random.default_rng(7)
    for r_bump in (0.4, 1.5, 3.3, 12.0):
        thr = np.float32(np.float32(r_bump) ** 2 + np.float32(MARGIN))
        T = threshold(thr)
        assert T < I32_MAX
        dist = np.sqrt(np.float64(thr)) + 0.03
        zi, ri, zj, rj = _pairs(rng, 50000, 60.0, 60.0, dist)
        qb = quant_bound(pack(zi, ri), pack(zj, rj))
        assert (qb > T).all(), (r_bump, int((qb <= T).sum()))


def test_threshold_saturates_to_keep_everything():
    # r_bump above ~181 A: every quantised bound (<= 2^31 - 1) passes
    assert threshold(np.float32(182.0 ** 2)) == I32_MAX
    # the largest bound two packed atoms can have (|r| >= 0, so dr > -32768)
    far = quant_bound((np.array([-32768]), np.array([0])), (np.array([32767]), np.array([32767])))
    assert far[0] == 2**30 + 32767**2 and far[0] <= threshold(np.float32(182.0 ** 2))
    # and below it the integer threshold stays exact to the widening
    t = threshold(np.float32(9.0 + MARGIN))
    assert (3.0 * UNITS) ** 2 < t <= (np.sqrt(9.0 + MARGIN) * UNITS + 3.0) ** 2 + 1
