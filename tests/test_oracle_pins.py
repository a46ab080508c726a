"""Pins for the FP64 oracle against facts fixed by mathematics, not by itself.

Each test names what pins it: closed forms of the 12-6 law (its minimum at
2^(1/6) sigma with depth eps, its zero at sigma, F = -du/dr), Newton's
third law (section 2.1), exact lattice symmetry, invariance under
translation and relabelling, brute force on tiny inputs, time reversal of
velocity Verlet, finite differences for the network gradient and
hand-derived values (tests/golden/).
"""
import json
import math
import os

import numpy as np
import pytest

from paper_2512_03565_amd import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def frms(f):
    return float(np.sqrt((f * f).sum(1).mean()))


# ---------------------------------------------------------------- pair law

@pytest.mark.parametrize("eps,sig", [(1.0, 1.0), (0.8, 1.2), (2.5, 0.7)])
def test_pair_minimum_and_zero_crossing(orc, eps, sig):
    # minimum of the 12-6 well at r = 2^(1/6) sigma: zero force, u = -eps
    rmin = 2.0 ** (1.0 / 6.0) * sig
    f, u, w = orc.lj_pair(rmin * rmin, eps, sig, rc=10 * sig, shift=False)
    assert abs(f * rmin) < 1e-13 * eps / sig
    assert abs(u + eps) < 1e-14 * max(1, eps)
    assert abs(w) < 1e-13 * eps
    # zero crossing at r = sigma, where |F| = -du/dr = 24 eps / sigma
    f, u, w = orc.lj_pair(sig * sig, eps, sig, rc=10 * sig, shift=False)
    assert abs(u) < 1e-14 * eps
    assert f * sig == pytest.approx(24.0 * eps / sig, rel=1e-14)
    assert w == pytest.approx(24.0 * eps, rel=1e-14)


def test_pair_long_range_tail(orc):
    # far from the core u -> -4 eps (sigma/r)^6 (the 12 term is 1e-6 of it at r = 10 sigma)
    r = 10.0
    _, u, _ = orc.lj_pair(r * r, 1.0, 1.0, rc=20.0, shift=False)
    assert u == pytest.approx(-4.0 * r ** -6, rel=2e-6)


@pytest.mark.parametrize("r", [0.92, 1.0, 1.1, 1.5, 2.2, 2.49])
def test_pair_force_is_minus_du_dr(orc, r):
    # the force magnitude along d is F . d / r = fscal * r, and must equal -du/dr
    h = 1e-6
    _, up, _ = orc.lj_pair((r + h) ** 2, 0.8, 1.2, rc=3.0, shift=False)
    _, um, _ = orc.lj_pair((r - h) ** 2, 0.8, 1.2, rc=3.0, shift=False)
    f, _, w = orc.lj_pair(r * r, 0.8, 1.2, rc=3.0, shift=False)
    dudr = (up - um) / (2 * h)
    assert f * r == pytest.approx(-dudr, rel=1e-7, abs=1e-9)
    # pair virial r . F = r * |F| (signed) = -r du/dr
    assert w == pytest.approx(-r * dudr, rel=1e-7, abs=1e-9)


def test_energy_shift(orc):
    rc = 2.5
    # shifted energy vanishes at the cutoff
    _, u, _ = orc.lj_pair((rc * (1 - 1e-12)) ** 2, 1.0, 1.0, rc=rc, shift=True)
    assert abs(u) < 1e-12
    # the shift is a constant offset equal to the unshifted u(rc)
    _, u_rc, _ = orc.lj_pair(rc * rc, 1.0, 1.0, rc=rc, shift=False)
    for r in (1.0, 1.7, 2.3):
        _, us, _ = orc.lj_pair(r * r, 1.0, 1.0, rc=rc, shift=True)
        _, un, _ = orc.lj_pair(r * r, 1.0, 1.0, rc=rc, shift=False)
        assert us - un == pytest.approx(-u_rc, rel=1e-12)


def two_particles(r, box=8.0, axis=0, t=(0, 0)):
    pos = np.array([[1.0, 1.5, 2.0], [1.0, 1.5, 2.0]])
    pos[1, axis] += r
    return pos, np.array([box, box, box]), np.array(t, np.int32)


@pytest.mark.parametrize("method", ["brute", "lc"])
def test_two_particle_system(orc, method):
    rmin = 2.0 ** (1.0 / 6.0)
    for axis in range(3):
        pos, box, _ = two_particles(1.0, axis=axis)
        res = orc.forces(pos, box, 2.5, shift=False, method=method)
        f = res["f"]
        # exact antisymmetry (Newton's third law, section 2.1)
        assert np.array_equal(f[0], -f[1])
        # at r = sigma: |F| = 24, pointing apart; U = u(sigma) = 0; W = r . F = 24
        assert f[1, axis] == pytest.approx(24.0, rel=1e-14)
        assert abs(res["U"]) < 1e-14 and res["W"] == pytest.approx(24.0, rel=1e-14)
        pos, box, _ = two_particles(rmin, axis=axis)
        res = orc.forces(pos, box, 2.5, shift=False, method=method)
        assert np.abs(res["f"]).max() < 1e-13
        assert res["U"] == pytest.approx(-1.0, rel=1e-14)
        assert res["u_i"] == pytest.approx([-0.5, -0.5], rel=1e-14)


def test_two_particles_across_periodic_boundary(orc):
    # separation r through the boundary: x = 0.3 and x = L - 0.7 are 1.0 apart
    box = np.array([8.0, 8.0, 8.0])
    pos = np.array([[0.3, 4.0, 4.0], [7.3, 4.0, 4.0]])
    for method in ("brute", "lc"):
        res = orc.forces(pos, box, 2.5, shift=False, method=method)
        assert res["f"][0, 0] == pytest.approx(24.0, rel=1e-12)
        assert res["f"][1, 0] == pytest.approx(-24.0, rel=1e-12)


def test_cutoff_is_strict(orc):
    # a pair at exactly r = rc does not interact; just inside it does
    box = np.array([8.0, 8.0, 8.0])
    pos = np.array([[1.0, 1.0, 1.0], [3.5, 1.0, 1.0]])  # r = 2.5 exactly
    for method in ("brute", "lc"):
        res = orc.forces(pos, box, 2.5, method=method)
        assert np.all(res["f"] == 0) and res["U"] == 0 and res["W"] == 0
    pos[1, 0] = np.nextafter(3.5, 0.0)
    res = orc.forces(pos, box, 2.5, method="lc")
    assert res["f"][0, 0] != 0


# ---------------------------------------------------------------- pair sums

def _random_systems():
    yield scenes.random_box(300, [9.0, 10.0, 11.0], seed=5), np.array([9.0, 10.0, 11.0]), None
    p, b = scenes.sc_lattice(8, 8, 8, 1.08, 0.05, seed=6)
    yield p, b, None
    p, b = scenes.fcc_lattice(6, 6, 6, 0.75, 0.05, seed=7)
    yield p, b, scenes.random_species(len(p), 2, seed=8)


@pytest.mark.parametrize("k", [0, 1, 2])
def test_brute_equals_linked_cells(orc, k):
    pos, box, types = list(_random_systems())[k]
    # random boxes have overlapping particles: keep r >= 0.8 sigma off the table
    eps, sig = ([1.0, 0.8], [1.0, 1.2]) if types is not None else (1.0, 1.0)
    rc = 2.5 if types is None else 3.0
    a = orc.forces(pos, box, rc, eps, sig, types, method="brute")
    b = orc.forces(pos, box, rc, eps, sig, types, method="lc")
    scale = max(frms(a["f"]), 1.0)
    assert np.abs(a["f"] - b["f"]).max() <= 1e-12 * scale * 100
    assert b["U"] == pytest.approx(a["U"], rel=1e-12)
    assert b["W"] == pytest.approx(a["W"], rel=1e-12)
    assert np.allclose(a["u_i"], b["u_i"], rtol=1e-11, atol=1e-11)


def test_pair_count_matches_numpy_brute_force(orc):
    pos, box = scenes.fcc_lattice(5, 5, 6, 0.75, 0.05, seed=9)
    d = pos[:, None, :] - pos[None, :, :]
    d -= box * np.rint(d / box)
    r2 = (d * d).sum(-1)
    iu = np.triu_indices(len(pos), 1)
    expect = int((r2[iu] < 2.8 ** 2).sum())
    pi, pj, pr2 = orc.pairs_within(pos, box, 2.8)
    assert len(pi) == expect
    assert np.all(pi < pj)
    assert np.allclose(pr2, r2[pi, pj], rtol=0, atol=1e-12)


def test_newton3_total_force_vanishes(orc):
    pos, box = scenes.fcc_lattice(8, 8, 8, 0.75, 0.05, seed=10)
    res = orc.forces(pos, box, 2.5)
    tot = res["f"].sum(0)
    assert np.abs(tot).max() <= 1e-11 * frms(res["f"]) * math.sqrt(len(pos))


@pytest.mark.parametrize("lattice", ["fcc", "sc"])
def test_perfect_lattice_symmetry(orc, lattice):
    # every site of a perfect periodic lattice is equivalent: zero net force, equal energies
    if lattice == "fcc":
        pos, box = scenes.fcc_lattice(6, 6, 6, 0.75)
    else:
        pos, box = scenes.sc_lattice(8, 8, 8, 1.08)
    res = orc.forces(pos, box, 2.5, method="lc")
    assert np.abs(res["f"]).max() < 1e-11
    assert np.ptp(res["u_i"]) < 1e-12
    assert res["U"] == pytest.approx(res["u_i"].sum(), rel=1e-13)


def test_translation_and_permutation_invariance(orc):
    pos, box = scenes.fcc_lattice(6, 6, 6, 0.75, 0.05, seed=11)
    ref = orc.forces(pos, box, 2.5)
    rng = np.random.default_rng(12)
    shift = rng.uniform(-50, 50, 3)
    perm = rng.permutation(len(pos))
    moved = (pos + shift)[perm]
    moved -= box * np.floor(moved / box)
    got = orc.forces(moved, box, 2.5)
    scale = frms(ref["f"])
    assert np.abs(got["f"] - ref["f"][perm]).max() < 1e-11 * scale
    assert got["U"] == pytest.approx(ref["U"], rel=1e-12)
    assert got["W"] == pytest.approx(ref["W"], rel=1e-12)


def test_two_equal_species_equal_one_species(orc):
    pos, box = scenes.fcc_lattice(5, 5, 5, 0.75, 0.05, seed=13)
    types = scenes.random_species(len(pos), 2, seed=14)
    one = orc.forces(pos, box, 2.5, 1.3, 0.9)
    two = orc.forces(pos, box, 2.5, [1.3, 1.3], [0.9, 0.9], types)
    assert np.abs(one["f"] - two["f"]).max() < 1e-13 * frms(one["f"])
    assert two["U"] == pytest.approx(one["U"], rel=1e-14)


def test_mixed_pair_special_point(orc):
    # Lorentz-Berthelot: sigma_ab = 1.1, eps_ab = sqrt(0.8); minimum at 2^(1/6) * 1.1
    rmin = 2.0 ** (1.0 / 6.0) * 1.1
    pos, box, types = two_particles(rmin, box=9.0, t=(0, 1))
    res = orc.forces(pos, box, 3.0, [1.0, 0.8], [1.0, 1.2], types, shift=False)
    assert np.abs(res["f"]).max() < 1e-13
    assert res["U"] == pytest.approx(-math.sqrt(0.8), rel=1e-14)
    # zero crossing at r = sigma_ab with |F| = 24 eps_ab / sigma_ab
    pos, box, types = two_particles(1.1, box=9.0, t=(1, 0))
    res = orc.forces(pos, box, 3.0, [1.0, 0.8], [1.0, 1.2], types, shift=False, method="brute")
    assert res["f"][1, 0] == pytest.approx(24 * math.sqrt(0.8) / 1.1, rel=1e-14)


def test_cell_binning_places_particles_in_their_cells(orc):
    pos, box = scenes.fcc_lattice(7, 7, 11, 0.75, 0.05, seed=15)
    nc = np.array([orc.ncell(b, 2.5) for b in box])
    cells = orc.bin_cells(pos, box, nc)
    cz, rem = np.divmod(cells, nc[0] * nc[1])
    cy, cx = np.divmod(rem, nc[0])
    c = np.stack([cx, cy, cz], 1)
    edge = box / nc
    assert np.all(pos >= c * edge - 1e-12) and np.all(pos <= (c + 1) * edge + 1e-12)
    assert np.all(edge >= 2.5)


def test_subset_matches_full(orc):
    pos, box = scenes.fcc_lattice(6, 6, 6, 0.75, 0.05, seed=16)
    full = orc.forces(pos, box, 2.5)
    idx = np.array([0, 5, 17, 300, len(pos) - 1])
    sub = orc.forces_subset(pos, box, 2.5, idx)
    assert np.array_equal(sub["f"], full["f"][idx])


# ---------------------------------------------------------------- dynamics

def test_velocity_verlet_energy_and_time_reversal(orc):
    s = scenes.config1()
    pos, vel, f, ep, ek = orc.vv(s["pos"], s["vel"], s["box"], s["rc"], s["dt"], 10)
    e = ep + ek
    assert np.abs(e - e[0]).max() / abs(e[0]) <= 1e-4
    # velocity Verlet is time reversible: flip v, integrate back, arrive at the start
    pos2, vel2, _, _, _ = orc.vv(pos, -vel, s["box"], s["rc"], s["dt"], 10)
    d = pos2 - s["pos"]
    d -= s["box"] * np.rint(d / s["box"])
    assert np.abs(d).max() < 1e-10
    assert np.abs(vel2 + s["vel"]).max() < 1e-9


def test_velocity_verlet_mass_scaling(orc):
    # Velocity Verlet with mass m, step dt and start velocities v0 visits the
    # same positions as mass 1, step dt/sqrt(m) and velocities v0 sqrt(m):
    # both kicks change v by F dt/(2m) = sqrt(m) F (dt/sqrt(m))/2 scaled
    # back by sqrt(m), and both drifts move x by dt v (section 2.1 names the
    # integrator; the identity is exact in real arithmetic).  Velocities
    # differ by the factor sqrt(m), kinetic energies not at all.  A kick
    # that multiplied by m, or missed the mass, fails this.
    s = scenes.config1()
    m = 2.5
    r = math.sqrt(m)
    pa, va, fa, epa, eka = orc.vv(s["pos"], s["vel"], s["box"], s["rc"], s["dt"], 10, mass=m)
    pb, vb, fb, epb, ekb = orc.vv(s["pos"], s["vel"] * r, s["box"], s["rc"], s["dt"] / r, 10,
                                  mass=1.0)
    d = pa - pb
    d -= s["box"] * np.rint(d / s["box"])
    assert np.abs(d).max() < 1e-12
    assert np.abs(va * r - vb).max() < 1e-11
    assert np.allclose(eka, ekb, rtol=1e-12, atol=0)
    assert np.allclose(epa, epb, rtol=1e-12, atol=0)
    # and the mass does change the trajectory
    pc, _, _, _, _ = orc.vv(s["pos"], s["vel"], s["box"], s["rc"], s["dt"], 10, mass=1.0)
    d = pa - pc
    d -= s["box"] * np.rint(d / s["box"])
    assert np.abs(d).max() > 1e-6


def test_velocity_verlet_two_masses_conserve_momentum_and_energy(orc):
    # Two species of masses 1 and 2.5.  Pair forces cancel (Newton's third
    # law, section 2.1), so each kick adds sum_i m_i (F_i dt / 2 m_i) = 0 to
    # the total momentum: it stays at its start value, zero, to rounding.  A
    # kick that used one species' mass for all particles would change it by
    # sum_i (m_i / m_used - 1) F_i dt / 2.  The kinetic energy is
    # 1/2 sum m_i v_i^2 at the start, and E = U + K stays near its start.
    s = scenes.config4(ncell=6)
    types = s["types"]
    masses = np.array([1.0, 2.5])
    mi = masses[types]
    v0 = scenes.mb_velocities(len(types), 1.0, mi, seed=83)
    p, v, f, ep, ek = orc.vv(s["pos"], v0, s["box"], s["rc"], s["dt"], 20, s["eps"], s["sig"],
                             mass=masses, types=types)
    scale = (mi[:, None] * np.abs(v)).sum()
    assert np.abs((mi[:, None] * v0).sum(0)).max() < 1e-13 * scale
    assert np.abs((mi[:, None] * v).sum(0)).max() < 1e-12 * scale
    assert ek[0] == pytest.approx(0.5 * (mi[:, None] * v0 * v0).sum(), rel=1e-14)
    e = ep + ek
    assert np.abs(e - e[0]).max() / abs(e[0]) <= 1e-4
    # with the masses swapped the same start moves differently
    p2, v2, _, _, _ = orc.vv(s["pos"], v0, s["box"], s["rc"], s["dt"], 20, s["eps"], s["sig"],
                             mass=masses[::-1].copy(), types=types)
    assert np.abs((mi[:, None] * v2).sum(0)).max() > 1e-6 * scale


# ---------------------------------------------------------------- network

def test_mlp_forward_golden(orc):
    g = json.load(open(os.path.join(GOLDEN, "mlp_tiny.json")))
    params = [np.array(g[k]) for k in ("W1", "b1", "W2", "b2", "W3", "b3")]
    h1, h2, z, p = orc.mlp_forward(params, np.array([g["x"]]))
    assert np.allclose(h1[0], g["h1"], rtol=0, atol=1e-15)
    assert np.allclose(h2[0], g["h2"], rtol=0, atol=1e-15)
    assert np.allclose(z[0], g["logits"], rtol=0, atol=1e-15)
    assert np.allclose(p[0], g["probs"], rtol=1e-15, atol=0)
    loss, _ = orc.mlp_loss_grad(params, np.array([g["x"]]), [g["label"]])
    assert loss == pytest.approx(g["loss"], rel=1e-15)


def _rand_params(rng, dims):
    ps = []
    for a, b in zip(dims[:-1], dims[1:]):
        ps += [rng.normal(0, 0.7, (b, a)), rng.normal(0, 0.3, b)]
    return ps


def test_mlp_gradient_matches_finite_differences(orc):
    rng = np.random.default_rng(17)
    params = _rand_params(rng, [8, 6, 5, 4])
    X = rng.normal(0, 1, (5, 8))
    y = rng.integers(0, 4, 5)
    _, grads = orc.mlp_loss_grad(params, X, y)
    h = 1e-6
    worst = 0.0
    for p, g in zip(params, grads):
        flat = p.reshape(-1)
        for k in range(flat.size):
            old = flat[k]
            flat[k] = old + h
            lp, _ = orc.mlp_loss_grad(params, X, y)
            flat[k] = old - h
            lm, _ = orc.mlp_loss_grad(params, X, y)
            flat[k] = old
            fd = (lp - lm) / (2 * h)
            worst = max(worst, abs(fd - g.reshape(-1)[k]) / max(abs(fd), 1e-3))
    assert worst < 1e-6


def test_adam_first_step_closed_form(orc):
    # after one step from zero moments the bias-corrected ratio is g/|g|:
    # w1 = w0 - lr * g / (|g| + eps)
    rng = np.random.default_rng(18)
    w = rng.normal(0, 1, 20)
    g = rng.normal(0, 1, 20)
    w0 = w.copy()
    m = np.zeros(20)
    v = np.zeros(20)
    orc.adam_step(w, g, m, v, 1, lr=1e-2, eps=1e-8)
    assert np.allclose(w, w0 - 1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-13, atol=1e-15)
    # a constant gradient keeps the bias-corrected ratio at g/|g| on later steps
    for t in range(2, 6):
        prev = w.copy()
        orc.adam_step(w, g, m, v, t, lr=1e-2, eps=1e-8)
        assert np.allclose(prev - w, 1e-2 * np.sign(g), rtol=1e-6)


# ---------------------------------------------------------------- inputs

def test_poisson_disk_droplet_spacing_and_counts():
    # the droplet workload's sampler: exact counts inside and outside the
    # sphere, and no two points (periodic) closer than the spacing
    from scipy.spatial import cKDTree
    pos, box = scenes.droplet_scene(20_000, 10.0, 0.8, 0.05, 0.9, seed=7)
    c = box / 2
    inside = ((pos - c) ** 2).sum(1) < 100.0
    assert inside.sum() == int(round(0.8 * 4.0 / 3.0 * math.pi * 1000.0))
    assert len(pos) == 20_000
    tree = cKDTree(pos, boxsize=box)
    assert len(tree.query_pairs(0.9 * (1 - 1e-12))) == 0
