"""Parity metrics between the HIP path and the FP64 oracle.

Force error norm (per particle, normalised so that particles whose net
force nearly cancels are not over-weighted):

    err_F = max_i ||F_i - F_i^ref|| / max(||F_i^ref||, F_rms^ref)

Pairs whose squared distance sits within a few ulps of rc^2 may be counted
inside the cutoff by one arithmetic and outside by the other; both answers
are correct for that arithmetic.  For the particles of such pairs the
allowed deviation is the summed magnitude of those pair forces (and
energies/virials for the totals), computed by the oracle.
"""
from __future__ import annotations

import numpy as np

F32_BAND = 4 * 2.0 ** -24
F64_BAND = 4 * 2.0 ** -53

# Words of the fixed-point frame of the FP32-pair staged kernel lie within
# this many grid steps of the box centre (the library's frame rule).
FX_RANGE = 1.5 * 2.0 ** 30


def fx_step(box, rc, skin):
    """Grid step 1/s of the fixed-point words for a box: s = FX_RANGE / reach,
    reach = the largest half edge plus one halo cell (edge L / floor(L /
    (rc + skin))) plus rc + skin."""
    rl = rc + skin
    reach = max(0.5 * L + L / np.floor(L / rl) for L in np.asarray(box, np.float64)) + rl
    return reach / FX_RANGE


def fx_band(box, rc, skin):
    """Cutoff band of the FP32-pair staged kernel.  It decides r^2 < rc^2 on
    the exact separation of coordinates rounded to the grid 1/s (at most half
    a step each), so its r^2 differs from the oracle's by at most
    2 |d| sqrt(3) step + 3 step^2: relative to rc^2, 2 sqrt(3) step / rc
    (plus rounding of r^2).  Never narrower than the FP32 band."""
    step = fx_step(box, rc, skin)
    return max(F32_BAND, (2 * np.sqrt(3) * step / rc + 3 * (step / rc) ** 2) * (1 + 1e-6)
               + 4 * 2.0 ** -53)


def list_band(box, rl):
    """Band of (rc + skin)^2 in which the list builds may decide a pair
    differently from the oracle: both form d in FP64, the builds from halo
    images at x +- L (one rounding of at most half an ulp of L), the oracle
    by the minimum image of x_i - x_j (another); |d| <= rl per axis gives
    |d(r^2)| <= 2 sqrt(3) rl ulp(L), relative 2 sqrt(3) ulp(L) / rl, doubled,
    plus a few roundings of r^2."""
    return 4 * np.sqrt(3) * float(np.spacing(np.max(np.asarray(box, np.float64)))) / rl + \
        8 * 2.0 ** -53


def frms(f):
    return float(np.sqrt((f * f).sum(1).mean())) if len(f) else 0.0


def boundary_slack(orc, pos, box, rc, eps, sig, types, shift, band):
    """Per-particle force slack and total (U, W) slack from pairs within the
    ambiguous band |r^2/rc^2 - 1| <= band."""
    n = len(pos)
    slack = np.zeros(n)
    su = sw = 0.0
    namb = 0
    pi, pj, r2 = orc.pairs_within(pos, box, rc * np.sqrt(1.0 + 2 * band))
    sel = np.abs(r2 / (rc * rc) - 1.0) <= band
    eps = np.atleast_1d(eps)
    sig = np.atleast_1d(sig)
    for a, b, q in zip(pi[sel], pj[sel], r2[sel]):
        ta = 0 if types is None else int(types[a])
        tb = 0 if types is None else int(types[b])
        e_ab, s_ab = orc.mix(eps[ta], sig[ta], eps[tb], sig[tb])
        f, u, w = orc.lj_pair(q, e_ab, s_ab, rc, shift)
        mag = abs(f) * np.sqrt(q) * (1 + 1e-6)
        slack[a] += mag
        slack[b] += mag
        su += abs(u) * (1 + 1e-6)
        sw += abs(w) * (1 + 1e-6)
        namb += 1
    return slack, su, sw, namb


def force_error(f, ref, slack=None, idx=None, scale=None):
    """err_F over the particles idx (all if None); scale overrides F_rms."""
    d = np.linalg.norm(np.asarray(f) - np.asarray(ref), axis=1)
    if slack is not None:
        d = np.maximum(0.0, d - slack)
    nr = np.linalg.norm(ref, axis=1)
    s = frms(ref) if scale is None else scale
    if len(d) == 0:
        return 0.0
    return float((d / np.maximum(nr, s)).max())


def total_error(val, ref, slack=0.0):
    return max(0.0, abs(val - ref) - slack) / max(abs(ref), 1e-300)


def boundary_slack_subset(orc, pos, box, rc, eps, sig, types, shift, band, idx):
    """Force slack of the particles idx only (for large scenes): their pairs
    in the ambiguous band, found with a periodic k-d tree; r^2 is formed as
    the oracle forms it (minimum image, then dx*dx + dy*dy + dz*dz)."""
    from scipy.spatial import cKDTree
    box = np.asarray(box, np.float64)
    w = pos - box * np.floor(pos / box)
    w = np.where(w >= box, w - box, w)
    tree = cKDTree(w, boxsize=box)
    eps = np.atleast_1d(eps)
    sig = np.atleast_1d(sig)
    slack = np.zeros(len(idx))
    hits = tree.query_ball_point(w[idx], rc * np.sqrt(1.0 + 2 * band) * (1 + 1e-9))
    for q, (a, js) in enumerate(zip(idx, hits)):
        if not js:
            continue
        js = np.asarray(js)
        js = js[js != a]
        d = pos[a] - pos[js]
        d -= box * np.rint(d / box)
        r2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
        for b, r2b in zip(js[np.abs(r2 / (rc * rc) - 1.0) <= band],
                          r2[np.abs(r2 / (rc * rc) - 1.0) <= band]):
            ta = 0 if types is None else int(types[a])
            tb = 0 if types is None else int(types[b])
            e_ab, s_ab = orc.mix(eps[ta], sig[ta], eps[tb], sig[tb])
            f, _, _ = orc.lj_pair(float(r2b), e_ab, s_ab, rc, shift)
            slack[q] += abs(f) * np.sqrt(r2b) * (1 + 1e-6)
    return slack
