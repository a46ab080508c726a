"""GPU parity of the linked-cell force kernels against the FP64 oracle.

Every linked-cell configuration (i-per-lane with i-tiles of 1/2/4 cells,
cluster tiles 8x8 and 16x4, wave-per-i with 1/2/4 i's per wavefront) in
both arithmetics, on seeded scenes that span many cells and have ragged
cell occupancies.  Tolerances: 1e-12 (all-FP64) and 1e-5 (FP32 pair
arithmetic, FP64 accumulation) in the per-particle norm of tests/_parity.py.
"""
import numpy as np
import pytest

from paper_2512_03565_amd import scenes
from tests import _parity as P

pytestmark = pytest.mark.gpu

TOL = {0: 1e-5, 1: 1e-12}


@pytest.fixture(scope="module")
def m():
    from paper_2512_03565_amd import mdlj
    return mdlj


def lc_configs(m):
    out = [(m.NBR_LC, m.ORD_I_PER_LANE, k, 1, 0, 0, 0) for k in (1, 2, 4)]
    for st in (0, 1):
        out += [(m.NBR_LC, m.ORD_CLUSTER_TILE, a, 64 // a, 0, 0, st) for a in (8, 16)]
        out += [(m.NBR_LC, m.ORD_WAVE_PER_I, g, 64 // g, 0, 0, st) for g in (1, 2, 4)]
    return out + lc_n3_configs(m)


def lc_n3_configs(m):
    """Newton 3 over a half shell of cells: the own particles as the i-list
    (three lane grids) and the roles swapped."""
    return [(m.NBR_LC, m.ORD_WAVE_PER_I, 1, 64, 0, 1, 1, 0),
            (m.NBR_LC, m.ORD_CLUSTER_TILE, 4, 16, 0, 1, 1, 0),
            (m.NBR_LC, m.ORD_CLUSTER_TILE, 16, 4, 0, 1, 1, 0),
            (m.NBR_LC, m.ORD_I_PER_LANE, 1, 1, 0, 1, 1, 1)]


def check_scene(m, orc, s, configs, precs=(0, 1), label=""):
    pos, box, rc = s["pos"], s["box"], s["rc"]
    types = s["types"] if len(s["eps"]) > 1 else None
    ref = orc.forces(pos, box, rc, s["eps"], s["sig"], types, method="lc")
    with m.System(pos, box, rc, s["eps"], s["sig"], types=types) as sysm:
        for prec in precs:
            sysm.set_precision(prec)
            band = P.F32_BAND if prec == 0 else P.F64_BAND
            slack, su, sw, namb = P.boundary_slack(orc, pos, box, rc, s["eps"], s["sig"], types,
                                                   True, band)
            for cfg in configs:
                print(f"[lc parity] {label} prec={prec} cfg={cfg}", flush=True)
                sysm.set_config(cfg)
                f, U, W = sysm.forces()
                e = P.force_error(f, ref["f"], slack)
                assert e <= TOL[prec], (cfg, prec, e, namb)
                assert P.total_error(U, ref["U"], su) <= TOL[prec], (cfg, prec, U, ref["U"])
                assert P.total_error(W, ref["W"], sw) <= TOL[prec], (cfg, prec, W, ref["W"])


def test_lc_config1_all_orders(m, orc):
    check_scene(m, orc, scenes.config1(), lc_configs(m), label="cfg1")


def test_lc_two_species(m, orc):
    s = scenes.config4(ncell=12)
    check_scene(m, orc, s, lc_configs(m), label="2-species")


def test_lc_config2_100k(m, orc):
    check_scene(m, orc, scenes.config2(), lc_configs(m), label="cfg2")


def test_lc_sparse_ragged_cells(m, orc):
    # low density: many empty cells and very uneven occupancy
    box = np.array([17.0, 13.0, 11.0])
    pos = scenes.random_box(150, box, seed=21)
    # keep the random gas free of overlaps closer than 0.8 sigma
    keep = [0]
    for k in range(1, len(pos)):
        d = pos[keep] - pos[k]
        d -= box * np.rint(d / box)
        if (d * d).sum(1).min() > 0.64:
            keep.append(k)
    s = dict(pos=pos[keep], box=box, rc=2.5, eps=[1.0], sig=[1.0], types=None)
    check_scene(m, orc, s, lc_configs(m), label="sparse")


def test_lc_two_particles_closed_form(m):
    # at r = sigma the force is 24 eps/sigma along the separation, U = u(sigma) - shift
    box = np.array([9.0, 9.0, 9.0])
    for prec in (0, 1):
        for axis in range(3):
            pos = np.array([[8.6, 0.2, 4.0], [8.6, 0.2, 4.0]])
            pos[1, axis] += 1.0  # crosses the periodic boundary along x
            with m.System(pos, box, 2.5, shift=False, precision=prec) as sysm:
                for cfg in lc_configs(m):
                    sysm.set_config(cfg)
                    f, U, W = sysm.forces()
                    tol = 1e-6 if prec == 0 else 1e-13
                    assert f[1, axis] == pytest.approx(24.0, rel=tol), cfg
                    assert f[0, axis] == pytest.approx(-24.0, rel=tol), cfg
                    assert abs(U) < 1e-5 and W == pytest.approx(24.0, rel=tol), cfg


def test_lc_single_particle_and_positions_outside_box(m, orc):
    box = np.array([8.0, 8.0, 8.0])
    with m.System(np.array([[3.0, 3.0, 3.0]]), box, 2.5) as sysm:
        f, U, W = sysm.forces()
        assert np.all(f == 0) and U == 0 and W == 0
    # positions given outside [0, L) are wrapped; results equal the wrapped scene
    pos, bx = scenes.fcc_lattice(5, 5, 5, 0.75, 0.05, seed=22)
    shifted = pos + np.array([3 * bx[0], -2 * bx[1], 0.5 * bx[2]])
    ref = orc.forces(pos, bx, 2.5)
    with m.System(shifted, bx, 2.5, precision=1) as sysm:
        f, U, W = sysm.forces()
        assert P.force_error(f, ref["f"]) < 1e-11
        assert U == pytest.approx(ref["U"], rel=1e-11)


def test_lc_perfect_lattice_has_zero_force(m):
    pos, box = scenes.fcc_lattice(6, 6, 6, 0.75)
    with m.System(pos, box, 2.5, precision=1) as sysm:
        for cfg in lc_configs(m):
            sysm.set_config(cfg)
            f, U, W = sysm.forces()
            assert np.abs(f).max() < 1e-11


def test_count_pairs_matches_oracle(m, orc):
    for s in (scenes.config1(), scenes.config4(ncell=10)):
        pi, pj, r2 = orc.pairs_within(s["pos"], s["box"], s["rc"])
        with m.System(s["pos"], s["box"], s["rc"], s["eps"], s["sig"]) as sysm:
            assert sysm.count_pairs() == len(pi)


def test_errors_geometry_state_nonfinite(m):
    pos, box = scenes.fcc_lattice(3, 3, 3, 0.75, 0.05, seed=23)  # L = 5.2 < 3 rc
    with m.System(pos, box, 2.5) as sysm:
        with pytest.raises(m.MdljError) as ei:
            sysm.forces()
        assert ei.value.status == -7
    pos, box = scenes.fcc_lattice(5, 5, 5, 0.75, 0.05, seed=24)
    with m.System(pos, box, 2.5) as sysm:
        bad = pos.copy()
        bad[7, 1] = np.inf
        with pytest.raises(m.MdljError) as ei:
            sysm.set_positions(bad)
        assert ei.value.status == -6
        # the context stays usable after a rejected call
        f, U, W = sysm.forces()
        assert np.isfinite(f).all()


def test_lc_newton3_three_cells_per_axis(m, orc):
    # 3 cells per axis: a cell's forward neighbours across the periodic
    # boundary are images of cells whose own forward shell reaches it too;
    # each pair must still be computed exactly once
    pos, box = scenes.sc_lattice(7, 7, 8, 1.1, 0.08, seed=23)
    assert all(int(L // 2.5) == 3 for L in box)
    s = dict(pos=pos, box=box, rc=2.5, eps=[1.0], sig=[1.0], types=None)
    check_scene(m, orc, s, lc_n3_configs(m), label="3 cells")


def test_lc_newton3_net_force_vanishes(m, orc):
    # Newton's third law: the computed forces sum to zero to rounding
    s = scenes.config2()
    with m.System(s["pos"], s["box"], s["rc"], precision=1) as sysm:
        for cfg in lc_n3_configs(m):
            sysm.set_config(cfg)
            f, U, W = sysm.forces()
            net = np.abs(f.sum(0)).max()
            assert net <= 1e-11 * P.frms(f) * np.sqrt(len(f)), (cfg, net)
