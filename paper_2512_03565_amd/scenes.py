"""Seeded synthetic particle scenes (inputs only; no force arithmetic).

Both the HIP path and the CPU oracle take their inputs from here, so this
module holds nothing of the method itself: lattices, jitter, species
assignment, Maxwell-Boltzmann velocities and random-sequential-addition
(Poisson-disk) droplets.  Every generator takes an explicit seed and uses
NumPy's PCG64.

A scene is a dict with keys
  pos   (n, 3) float64, wrapped into [0, L)
  box   (3,)   float64, orthorhombic periodic box edges
  types (n,)   int32 species index
  eps, sig, mass  per-species parameters (lists)
  rc, skin, rebuild_every, T, dt  physics and method settings
  name  short description
"""
from __future__ import annotations

import math

import numpy as np

FCC_BASIS = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]])


def _wrap(pos, box):
    return pos - box * np.floor(pos / box)


def sc_lattice(nx, ny, nz, spacing, jitter=0.0, seed=0):
    """Simple-cubic lattice of nx*ny*nz sites, uniform +-jitter per coordinate."""
    g = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"),
                 -1).reshape(-1, 3).astype(np.float64)
    box = np.array([nx, ny, nz], np.float64) * spacing
    pos = (g + 0.5) * spacing
    if jitter:
        rng = np.random.default_rng(seed)
        pos = pos + rng.uniform(-jitter, jitter, pos.shape)
    return _wrap(pos, box), box


def fcc_lattice(nx, ny, nz, rho, jitter=0.0, seed=0):
    """FCC lattice of nx*ny*nz unit cells (4 sites each) at number density rho."""
    a = (4.0 / rho) ** (1.0 / 3.0)
    g = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"),
                 -1).reshape(-1, 3).astype(np.float64)
    pos = ((g[:, None, :] + FCC_BASIS[None] + 0.25) * a).reshape(-1, 3)
    box = np.array([nx, ny, nz], np.float64) * a
    if jitter:
        rng = np.random.default_rng(seed)
        pos = pos + rng.uniform(-jitter, jitter, pos.shape)
    return _wrap(pos, box), box


def mb_velocities(n, T, mass=1.0, seed=0):
    """Maxwell-Boltzmann velocities: N(0, sqrt(T/m)) per component, zero total
    momentum, rescaled to temperature T with 3n-3 degrees of freedom."""
    rng = np.random.default_rng(seed)
    m = np.broadcast_to(np.asarray(mass, np.float64), (n,))
    v = rng.normal(0.0, 1.0, (n, 3)) * np.sqrt(T / m)[:, None]
    p = (m[:, None] * v).sum(0) / m.sum()
    v -= p
    if n > 1:
        ke2 = (m[:, None] * v * v).sum()
        v *= math.sqrt(T * (3 * n - 3) / ke2)
    return v


def random_species(n, nspec, seed=0):
    """Independent uniform species assignment (50/50 for two species)."""
    if nspec == 1:
        return np.zeros(n, np.int32)
    rng = np.random.default_rng(seed)
    return rng.integers(0, nspec, n).astype(np.int32)


def random_box(n, box, seed=0):
    """Uniformly random positions in a box (used for tiny brute-force checks)."""
    rng = np.random.default_rng(seed)
    box = np.asarray(box, np.float64)
    return rng.uniform(0.0, 1.0, (n, 3)) * box


def rsa_points(box, count, dmin, seed, inside=None, existing=None, region=None,
               batch=1 << 18, progress=None, max_batches=200000):
    """Random sequential addition (Poisson-disk darts): uniform darts, kept
    when no accepted point lies closer than dmin (periodic box);
    ``inside(p) -> bool mask`` restricts the region, ``region = (lo, hi)``
    the sub-box the darts are drawn in; ``existing`` points count as
    accepted.  Returns the new points (count, 3).

    Vectorised on a grid of cells of edge dmin / sqrt(3), which hold at most
    one point each: a batch of darts is tested against the accepted points
    of the 5 x 5 x 5 cells around it, then against the earlier darts of the
    same batch (a dart near an earlier surviving one is dropped, whether or
    not that one survives its own tests, so the batch keeps the minimum
    spacing; this drops slightly more darts than one-at-a-time addition)."""
    rng = np.random.default_rng(seed)
    box = np.asarray(box, np.float64)
    nc = np.maximum(np.floor(box / (dmin / math.sqrt(3.0))).astype(np.int64), 1)
    edge = box / nc
    ne = 0 if existing is None else len(existing)
    grid = np.full(int(nc[0] * nc[1] * nc[2]), -1, np.int64)
    store = np.empty((count + ne, 3))

    def cells(p):
        return np.minimum((p / edge).astype(np.int64), nc - 1)

    def lin(c):
        c = c % nc
        return c[..., 0] + nc[0] * (c[..., 1] + nc[1] * c[..., 2])

    if ne:
        ex = np.asarray(existing, np.float64)
        grid[lin(cells(ex))] = np.arange(ne)
        store[:ne] = ex
    npts = ne
    offs = np.array([(dx, dy, dz) for dz in range(-2, 3) for dy in range(-2, 3)
                     for dx in range(-2, 3)])
    gap = np.maximum(np.abs(offs) - 1, 0) * edge
    offs = offs[(gap ** 2).sum(1) < dmin * dmin]
    d2 = dmin * dmin
    lo, hi = (np.zeros(3), box) if region is None else (np.asarray(region[0], np.float64),
                                                          np.asarray(region[1], np.float64))
    nb = 0
    while npts - ne < count:
        nb += 1
        if nb > max_batches:
            raise RuntimeError("RSA did not reach the requested count")
        cand = lo + rng.uniform(0.0, 1.0, (batch, 3)) * (hi - lo)
        cand -= box * np.floor(cand / box)
        if inside is not None:
            cand = cand[inside(cand)]
        c = cells(cand)
        ok = grid[lin(c)] < 0
        cand, c = cand[ok], c[ok]
        for o in offs:
            if len(cand) == 0:
                break
            j = grid[lin(c + o)]
            hit = j >= 0
            if hit.any():
                d = cand[hit] - store[j[hit]]
                d -= box * np.rint(d / box)
                bad = np.zeros(len(cand), bool)
                bad[np.flatnonzero(hit)[(d * d).sum(1) < d2]] = True
                cand, c = cand[~bad], c[~bad]
        if len(cand) == 0:
            continue
        # one dart per cell (the first), then no dart near an earlier one
        L = lin(c)
        order = np.argsort(L, kind="stable")
        first = np.ones(len(cand), bool)
        sl = L[order]
        first[order[np.r_[False, sl[1:] == sl[:-1]]]] = False
        cand, c, L = cand[first], c[first], L[first]
        keep = np.ones(len(cand), bool)
        grid[L] = -(np.arange(len(cand)) + 2)
        for o in offs:
            if (o == 0).all():
                continue
            j = grid[lin(c + o)]
            m = j <= -2
            if m.any():
                k = -(j[m] + 2)
                me = np.flatnonzero(m)
                e = k < me
                me, k = me[e], k[e]
                d = cand[me] - cand[k]
                d -= box * np.rint(d / box)
                keep[me[(d * d).sum(1) < d2]] = False
        grid[L] = -1
        room = count - (npts - ne)
        cand, L = cand[keep][:room], L[keep][:room]
        grid[L] = np.arange(npts, npts + len(cand))
        store[npts:npts + len(cand)] = cand
        npts += len(cand)
        if progress is not None and nb % 50 == 0:
            progress(npts - ne, count)
    return store[ne:npts].copy()


def droplet_scene(n_total, r_drop, rho_drop, rho_vap, dmin, seed, progress=None):
    """Spherical droplet at rho_drop in vapour at rho_vap, periodic cube of
    edge (V_drop + N_vap / rho_vap)^(1/3); Poisson-disk darts (random
    sequential addition) with minimum spacing dmin, droplet first (darts
    drawn in its bounding cube), then vapour outside it."""
    v_drop = 4.0 / 3.0 * math.pi * r_drop ** 3
    n_drop = int(round(rho_drop * v_drop))
    n_vap = n_total - n_drop
    L = (v_drop + n_vap / rho_vap) ** (1.0 / 3.0)
    box = np.array([L, L, L])
    c = box / 2

    def in_drop(p):
        return ((p - c) ** 2).sum(1) < r_drop * r_drop

    def out_drop(p):
        return ~in_drop(p)

    drop = rsa_points(box, n_drop, dmin, seed, inside=in_drop, region=(c - r_drop, c + r_drop),
                      progress=progress)
    vap = rsa_points(box, n_vap, dmin, seed + 1, inside=out_drop, existing=drop,
                     progress=progress)
    return np.concatenate([drop, vap]), box


def lattice_droplet(n, rho_drop, frac_drop=0.2, rho_vap=0.05, jitter=0.05, seed=0):
    """About n particles: a sphere holding frac_drop of them at density
    rho_drop (jittered FCC cut to the sphere) in vapour at rho_vap (a simple
    cubic lattice of spacing rho_vap^(-1/3) jittered by a quarter spacing,
    points inside the sphere or within 1.0 of its surface removed), in a
    periodic cube.  Minimum spacing stays above ~0.8 sigma."""
    rng = np.random.default_rng(seed)
    n_drop = int(frac_drop * n)
    n_vap = n - n_drop
    v_drop = n_drop / rho_drop
    r_drop = (3.0 * v_drop / (4.0 * math.pi)) ** (1.0 / 3.0)
    L = (v_drop + n_vap / rho_vap) ** (1.0 / 3.0)
    L = max(L, 2.0 * r_drop + 8.0)
    box = np.array([L, L, L])
    c = box / 2
    a = (4.0 / rho_drop) ** (1.0 / 3.0)
    m = int(math.ceil(2 * r_drop / a)) + 1
    g = np.stack(np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij"),
                 -1).reshape(-1, 3).astype(np.float64)
    d = ((g[:, None, :] + FCC_BASIS[None]) * a).reshape(-1, 3)
    d = d - d.mean(0)
    d = d[(d * d).sum(1) < r_drop * r_drop] + c
    d = d + rng.uniform(-jitter, jitter, d.shape)
    sp = rho_vap ** (-1.0 / 3.0)
    k = max(1, int(L / sp))
    sp = L / k
    g = np.stack(np.meshgrid(np.arange(k), np.arange(k), np.arange(k), indexing="ij"),
                 -1).reshape(-1, 3).astype(np.float64)
    v = (g + 0.5) * sp + rng.uniform(-0.25 * sp, 0.25 * sp, g.shape)
    rr = np.sqrt(((v - c) ** 2).sum(1))
    v = v[rr > r_drop + 1.0]
    return _wrap(np.concatenate([d, v]), box), box


def _scene(pos, box, **kw):
    s = dict(pos=np.ascontiguousarray(pos, np.float64), box=np.asarray(box, np.float64))
    s.update(kw)
    n = len(s["pos"])
    s.setdefault("types", np.zeros(n, np.int32))
    s.setdefault("eps", [1.0])
    s.setdefault("sig", [1.0])
    s.setdefault("mass", [1.0])
    return s


def config1(seed=1001):
    """1,000 particles, 10x10x10 simple cubic, spacing 1.08 sigma, +-0.05 jitter,
    periodic cube, rc 2.5, FP64, T = 1.0, dt = 0.002."""
    pos, box = sc_lattice(10, 10, 10, 1.08, 0.05, seed)
    return _scene(pos, box, rc=2.5, skin=0.3, rebuild_every=10, T=1.0, dt=0.002,
                  vel=mb_velocities(len(pos), 1.0, 1.0, seed + 7),
                  name="1k simple-cubic rho~0.79 rc2.5")


def config2(seed=1002):
    """100,000 particles: 25x25x40 FCC unit cells at rho = 0.75, +-0.05 jitter,
    rc 2.5, skin 0.3, rebuild every 10 steps, T = 1.0."""
    pos, box = fcc_lattice(25, 25, 40, 0.75, 0.05, seed)
    return _scene(pos, box, rc=2.5, skin=0.3, rebuild_every=10, T=1.0, dt=0.002,
                  vel=mb_velocities(len(pos), 1.0, 1.0, seed + 7),
                  name="100k FCC rho0.75 rc2.5")


def headline(seed=20251203):
    """1,000,000 particles: 50x50x100 FCC unit cells at rho = 0.75 (box
    87.358 x 87.358 x 174.716), +-0.05 jitter, rc 2.5, skin 0.3, rebuild
    every 10 steps, T = 1.0."""
    pos, box = fcc_lattice(50, 50, 100, 0.75, 0.05, seed)
    return _scene(pos, box, rc=2.5, skin=0.3, rebuild_every=10, T=1.0, dt=0.002,
                  name="1M FCC rho0.75 rc2.5 skin0.3")


def config4(seed=1004, ncell=100):
    """Two species (sigma 1.0/1.2, eps 1.0/0.8, Lorentz-Berthelot), 50/50
    random, ncell^3 FCC unit cells at rho = 0.7 (4M at ncell = 100),
    rc = 2.5 * sigma_max = 3.0, +-0.05 jitter."""
    pos, box = fcc_lattice(ncell, ncell, ncell, 0.7, 0.05, seed)
    types = random_species(len(pos), 2, seed + 3)
    return _scene(pos, box, types=types, eps=[1.0, 0.8], sig=[1.0, 1.2], mass=[1.0, 1.0],
                  rc=3.0, skin=0.3, rebuild_every=10, T=1.0, dt=0.002,
                  name=f"{len(pos)} two-species FCC rho0.7 rc3.0")


def config3(seed=1003, n_total=1_000_000, r_drop=40.0, progress=None):
    """Droplet of radius r_drop at rho 0.8 inside vapour at rho 0.05 in a
    periodic cube (edge 251.87 for 1M particles), positions by Poisson-disk
    sampling (random sequential addition) with minimum spacing 0.9, droplet
    first; rc 3.0, T = 0.9, skin 0.3, lists rebuilt every 10 steps."""
    pos, box = droplet_scene(n_total, r_drop, 0.8, 0.05, 0.9, seed, progress=progress)
    return _scene(pos, box, rc=3.0, skin=0.3, rebuild_every=10, T=0.9, dt=0.002,
                  name=f"{len(pos)} droplet r{r_drop}")


def exploding_block(ncell=(50, 50, 100), rho=0.75, box_factor=3.0, T=5.0, seed=1006):
    """A dense block released into vacuum (the paper's exploding-liquid
    benchmark, with synthetic sizes): jittered FCC of ncell unit cells at
    density rho (1M particles by default), centred in a periodic box
    box_factor times its size along every axis, Maxwell-Boltzmann
    velocities at the high temperature T, so the block expands into the
    empty space and the particle density changes across the run; rc 2.5,
    skin 0.3, lists rebuilt every 10 steps (earlier when a particle moves
    more than skin/2)."""
    pos, blk = fcc_lattice(ncell[0], ncell[1], ncell[2], rho, 0.05, seed)
    box = box_factor * blk
    pos = pos + 0.5 * (box - blk)
    return _scene(pos, box, rc=2.5, skin=0.3, rebuild_every=10, T=T, dt=0.002,
                  name=f"{len(pos)} exploding block T{T}")


def tuning_scene(index, n_min=1e4, n_max=4e6):
    """Scene `index` of the learned-tuner sweep (seed 50000 + index): N
    log-uniform in [n_min, n_max], density uniform in [0.05, 1.0], cutoff
    uniform in [2.5, 3.5] sigma_max, one or two species, homogeneous (jittered
    FCC) or droplet (20% of N at that density in vapour at 0.05)."""
    seed = 50000 + index
    rng = np.random.default_rng(seed)
    n = int(round(10 ** rng.uniform(math.log10(n_min), math.log10(n_max))))
    rho = float(rng.uniform(0.05, 1.0))
    rc_fac = float(rng.uniform(2.5, 3.5))
    nspec = int(rng.integers(1, 3))
    droplet = bool(rng.integers(0, 2))
    if droplet and rho > 0.1:
        pos, box = lattice_droplet(n, rho, seed=seed + 1)
    else:
        m = max(2, int(round((n / 4.0) ** (1.0 / 3.0))))
        nz = max(2, int(round(n / (4.0 * m * m))))
        pos, box = fcc_lattice(m, m, nz, rho, 0.05, seed + 1)
        droplet = False
    sig = [1.0, 1.2][:nspec]
    eps = [1.0, 0.8][:nspec]
    types = random_species(len(pos), nspec, seed + 2)
    rc = rc_fac * max(sig)
    return _scene(pos, box, types=types, eps=eps, sig=sig, mass=[1.0] * nspec, rc=rc, skin=0.3,
                  rebuild_every=10, T=1.0, dt=0.002,
                  name=f"tune{index} n={len(pos)} rho={rho:.3f} rc={rc:.2f} "
                       f"ns={nspec} {'droplet' if droplet else 'homog'}",
                  rho=rho, droplet=droplet)


def homogeneous_scene(n, rho, rc, nspec, seed):
    """Jittered FCC block of about n particles at density rho (nearly cubic
    box), one or two species; used for tuner training scenes."""
    m = max(2, int(round((n / 4.0) ** (1.0 / 3.0))))
    nz = max(2, int(round(n / (4.0 * m * m))))
    pos, box = fcc_lattice(m, m, nz, rho, 0.05, seed)
    if nspec == 2:
        return _scene(pos, box, types=random_species(len(pos), 2, seed + 3), eps=[1.0, 0.8],
                      sig=[1.0, 1.2], mass=[1.0, 1.0], rc=rc, skin=0.3, rebuild_every=10,
                      T=1.0, dt=0.002, name="homog2")
    return _scene(pos, box, rc=rc, skin=0.3, rebuild_every=10, T=1.0, dt=0.002, name="homog")
