"""GPU parity of the Verlet-list kernels, the list upkeep between rebuilds
(refresh while every particle moved < skin/2, early rebuild otherwise) and
the velocity-Verlet integrator, against the FP64 oracle."""
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


def vl_configs(m):
    out = []
    for n3 in (0, 1):
        out.append((m.NBR_VL, m.ORD_I_PER_LANE, 0, 0, 0, n3))
        out += [(m.NBR_VL, m.ORD_WAVE_PER_I, g, 64 // g, 0, n3) for g in (1, 2, 4, 8, 16)]
    out += [(m.NBR_VL, m.ORD_WAVE_PER_I, g, v, 0, 0, 1) for g, v in ((8, 2), (8, 4), (16, 2),
                                                                      (16, 4), (4, 8))]
    return out


def check(m, orc, s, configs, label, precs=(0, 1), skin=0.3):
    pos, box, rc = s["pos"], s["box"], s["rc"]
    types = s["types"] if len(s["eps"]) > 1 else None
    ref = orc.forces(pos, box, rc, s["eps"], s["sig"], types)
    with m.System(pos, box, rc, s["eps"], s["sig"], types=types, skin=skin) as sysm:
        for prec in precs:
            sysm.set_precision(prec)
            band = P.fx_band(box, rc, skin) if prec == 0 else P.F64_BAND
            slack, su, sw, namb = P.boundary_slack(orc, pos, box, rc, s["eps"], s["sig"], types,
                                                   True, band)
            for cfg in configs:
                print(f"[vl parity] {label} prec={prec} cfg={cfg}", flush=True)
                sysm.set_config(cfg)
                f, U, W = sysm.forces()
                e = P.force_error(f, ref["f"], slack)
                print(f"[vl parity]   err_F {e:.3e}", flush=True)
                assert e <= TOL[prec], (cfg, prec, e, namb)
                assert P.total_error(U, ref["U"], su) <= TOL[prec], (cfg, prec, U, ref["U"])
                assert P.total_error(W, ref["W"], sw) <= TOL[prec], (cfg, prec, W, ref["W"])


def test_vl_config1(m, orc):
    check(m, orc, scenes.config1(), vl_configs(m), "cfg1")


def test_vl_two_species(m, orc):
    check(m, orc, scenes.config4(ncell=12), vl_configs(m), "2-species")


def test_vl_config2_100k(m, orc):
    check(m, orc, scenes.config2(), vl_configs(m), "cfg2")


def test_vl_dense_large_cells_fall_back(m, orc):
    # rc = 4: about 70 particles per cell.  The tiled list build cannot stage
    # a tile's neighbourhood in LDS, so the lists come from the per-particle
    # build.  The FP32-pair staged kernel still fits it (16-byte fixed-point
    # records, ~54 KB); the all-FP64 one (24 bytes and the species) does not
    # and is refused with MDLJ_ERR_ARG
    pos, box = scenes.fcc_lattice(8, 8, 8, 0.9, 0.05, seed=41)
    s = dict(pos=pos, box=box, rc=4.0, eps=[1.0], sig=[1.0], types=None)
    plain = [c for c in vl_configs(m) if len(c) < 7]
    staged = [c for c in vl_configs(m) if len(c) == 7]
    check(m, orc, s, plain, "dense")
    check(m, orc, s, staged, "dense", precs=(0,))
    with m.System(pos, box, 4.0, skin=0.3, precision=1) as sysm:
        for cfg in staged:
            with pytest.raises(m.MdljError) as ei:
                sysm.set_config(cfg)
                sysm.forces()
            assert ei.value.status == -1, cfg


def test_vl_zero_skin_equals_cutoff_lists(m, orc):
    check(m, orc, scenes.config1(), vl_configs(m)[:2], "skin0", skin=0.0)


def test_vl_refresh_and_early_rebuild(m, orc):
    s = scenes.config2()
    pos, box, rc = s["pos"], s["box"], s["rc"]
    rng = np.random.default_rng(31)
    with m.System(pos, box, rc, skin=0.3, rebuild_every=1000, precision=1) as sysm:
        for cfg in ((m.NBR_VL, m.ORD_I_PER_LANE, 0, 0, 0, 0),
                    (m.NBR_VL, m.ORD_WAVE_PER_I, 2, 32, 0, 1),
                    (m.NBR_VL, m.ORD_WAVE_PER_I, 16, 4, 0, 0, 1)):
            sysm.set_config(cfg)
            sysm.set_positions(pos)
            sysm.set_timing(True)
            sysm.forces()
            # small moves (< skin/2): records are refreshed, the lists kept
            moved = pos + rng.uniform(-0.08, 0.08, pos.shape)
            sysm.set_positions(moved)
            f, U, W = sysm.forces()
            _, _, nf, nb = sysm.get_timing()
            assert (nf, nb) == (2, 1), (cfg, nf, nb)
            ref = orc.forces(moved, box, rc)
            assert P.force_error(f, ref["f"]) <= 1e-12, cfg
            # one particle moves by 0.2 > skin/2: the lists must be rebuilt
            moved2 = moved.copy()
            moved2[123] = pos[123] + np.array([0.2, 0.0, 0.0])
            sysm.set_positions(moved2)
            f, U, W = sysm.forces()
            _, _, nf, nb = sysm.get_timing()
            assert (nf, nb) == (3, 2), (cfg, nf, nb)
            ref = orc.forces(moved2, box, rc)
            assert P.force_error(f, ref["f"]) <= 1e-12, cfg


@pytest.mark.parametrize("cfg", [(0, 0, 1, 1, 0, 0), (0, 2, 2, 32, 0, 0), (1, 0, 0, 0, 0, 0),
                                 (1, 2, 1, 64, 0, 1), (1, 2, 8, 2, 0, 0, 1), (0, 1, 16, 4, 0, 0, 1)])
def test_velocity_verlet_trajectory_matches_oracle(m, orc, cfg):
    import torch
    s = scenes.config1()
    p_ref, v_ref, f_ref, ep, ek = orc.vv(s["pos"], s["vel"], s["box"], s["rc"], s["dt"], 10)
    with m.System(s["pos"], s["box"], s["rc"], skin=0.3, rebuild_every=4, precision=1) as sysm:
        sysm.set_config(cfg)
        vel = [torch.tensor(np.ascontiguousarray(s["vel"][:, k]), device="cuda") for k in range(3)]
        sysm.step_vv(vel, s["dt"], 10)
        f, U, W = sysm.forces()
        pos = sysm.get_positions()
    v = torch.stack(vel, 1).cpu().numpy()
    d = pos - p_ref
    d -= s["box"] * np.rint(d / s["box"])
    assert np.abs(d).max() < 1e-10, cfg
    assert np.abs(v - v_ref).max() < 1e-9, cfg
    assert P.force_error(f, f_ref) < 1e-9, cfg
    assert U == pytest.approx(ep[-1], rel=1e-10)


@pytest.mark.parametrize("cfg", [(1, 2, 16, 4, 0, 0, 1), (1, 2, 4, 16, 0, 1)])
def test_velocity_verlet_fast_particles_force_early_rebuilds(m, orc, cfg):
    # velocities 15x thermal: particles cross skin/2 between scheduled
    # rebuilds, so the displacement test of the integrator must trigger them
    import torch
    s = scenes.config1()
    v0 = 15.0 * s["vel"]
    p_ref, v_ref, f_ref, ep, ek = orc.vv(s["pos"], v0, s["box"], s["rc"], s["dt"], 12)
    with m.System(s["pos"], s["box"], s["rc"], skin=0.3, rebuild_every=6, precision=1) as sysm:
        sysm.set_config(cfg)
        vel = [torch.tensor(np.ascontiguousarray(v0[:, k]), device="cuda") for k in range(3)]
        sysm.set_timing(True)
        sysm.step_vv(vel, s["dt"], 12)
        _, _, nf, nb = sysm.get_timing()
        pos = sysm.get_positions()
    assert nb >= 5, (cfg, nf, nb)  # the schedule alone gives at most 3
    v = torch.stack(vel, 1).cpu().numpy()
    d = pos - p_ref
    d -= s["box"] * np.rint(d / s["box"])
    assert np.abs(d).max() < 1e-10, cfg
    assert np.abs(v - v_ref).max() < 1e-8, cfg


@pytest.mark.parametrize("prec,cfg", [(0, (1, 2, 16, 4, 0, 0, 1)), (1, (1, 2, 16, 4, 0, 0, 1)),
                                      (0, (1, 2, 8, 4, 0, 0, 1)), (1, (1, 2, 8, 8, 0, 0)),
                                      (1, (1, 0, 0, 0, 0, 0))])
def test_velocity_verlet_one_call_equals_single_steps(m, prec, cfg):
    # Between Verlet-list rebuilds a multi-step call keeps the integrator
    # state in sorted order and writes it back before each rebuild and on
    # return (with the staged kernels the force kernel takes the integrator
    # step itself); one-step calls never enter that state.  The arithmetic is
    # the same, so 60 steps in one call and 60 calls of one step must agree
    # bit for bit, over six scheduled rebuilds and the displacement tests.
    import torch
    s = scenes.config2()
    n = len(s["pos"])
    v0 = scenes.mb_velocities(n, 1.0, 1.0, seed=77)
    out = []
    for single in (False, True):
        with m.System(s["pos"], s["box"], s["rc"], skin=0.3, rebuild_every=10,
                      precision=prec) as sysm:
            sysm.set_config(cfg)
            vel = [torch.tensor(np.ascontiguousarray(v0[:, k]), device="cuda") for k in range(3)]
            sysm.set_timing(True)
            if single:
                for _ in range(60):
                    sysm.step_vv(vel, s["dt"], 1)
            else:
                sysm.step_vv(vel, s["dt"], 60)
            _, _, nf, nb = sysm.get_timing()
            _, nfused = sysm.get_timing_fused()
            out.append((sysm.get_positions(), torch.stack(vel, 1).cpu().numpy(), nb, nfused))
    print(f"[vv one call vs single steps] prec={prec} cfg={cfg} rebuilds {out[0][2]} / {out[1][2]}"
          f", fused force calls {out[0][3]} / {out[1][3]}", flush=True)
    assert out[0][2] == out[1][2] >= 6, (cfg, out[0][2], out[1][2])
    # staged lists: every step of the call but the last and those before a
    # rebuild takes the integrator step inside the force kernel; one-step
    # calls never do
    staged = len(cfg) == 7 and cfg[6] == 1
    assert out[1][3] == 0
    assert (out[0][3] >= 60 - 1 - out[0][2]) if staged else out[0][3] == 0, out[0][3]
    assert np.array_equal(out[0][0], out[1][0]), cfg
    assert np.array_equal(out[0][1], out[1][1]), cfg


@pytest.mark.parametrize("prec", [0, 1])
def test_velocity_verlet_fused_step_two_species_two_masses_bitwise(m, prec):
    # The fused step picks 1/m by species; one-step calls use the separate
    # kick kernels, which index the mass table directly.  Two species of
    # different mass: one call of 30 steps equals 30 one-step calls bit for bit.
    import torch
    s = scenes.config4(ncell=12)
    n = len(s["pos"])
    v0 = scenes.mb_velocities(n, 1.0, 1.0, seed=81)
    cfg = (1, 2, 16, 4, 0, 0, 1)
    out = []
    for single in (False, True):
        with m.System(s["pos"], s["box"], s["rc"], s["eps"], s["sig"], types=s["types"],
                      skin=0.3, rebuild_every=10, precision=prec, mass=[1.0, 2.5]) as sysm:
            sysm.set_config(cfg)
            vel = [torch.tensor(np.ascontiguousarray(v0[:, k]), device="cuda") for k in range(3)]
            sysm.set_timing(True)
            if single:
                for _ in range(30):
                    sysm.step_vv(vel, s["dt"], 1)
            else:
                sysm.step_vv(vel, s["dt"], 30)
            _, nfused = sysm.get_timing_fused()
            out.append((sysm.get_positions(), torch.stack(vel, 1).cpu().numpy(), nfused))
    print(f"[fused step, two masses] prec={prec} fused calls {out[0][2]} / {out[1][2]}", flush=True)
    assert out[0][2] > 20 and out[1][2] == 0
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("cfg", [(1, 2, 16, 4, 0, 0, 1), (1, 0, 0, 0, 0, 0), (1, 2, 4, 16, 0, 1),
                                 (0, 0, 1, 1, 0, 0)])
def test_velocity_verlet_two_masses_match_oracle(m, orc, cfg):
    # Two species of masses 1 and 2.5 (mdlj_set_mass): 20 FP64 steps with
    # list rebuilds every 5 against the oracle's velocity Verlet with the
    # same per-species masses (section 2.1), at the trajectory bars of the
    # one-mass test.
    import torch
    s = scenes.config4(ncell=12)
    masses = np.array([1.0, 2.5])
    types = s["types"]
    v0 = scenes.mb_velocities(len(types), 1.0, masses[types], seed=85)
    p_ref, v_ref, f_ref, ep, ek = orc.vv(s["pos"], v0, s["box"], s["rc"], s["dt"], 20, s["eps"],
                                         s["sig"], mass=masses, types=types)
    with m.System(s["pos"], s["box"], s["rc"], s["eps"], s["sig"], types=types, skin=0.3,
                  rebuild_every=5, precision=1, mass=masses) as sysm:
        sysm.set_config(cfg)
        vel = [torch.tensor(np.ascontiguousarray(v0[:, k]), device="cuda") for k in range(3)]
        sysm.step_vv(vel, s["dt"], 20)
        f, U, W = sysm.forces()
        pos = sysm.get_positions()
    v = torch.stack(vel, 1).cpu().numpy()
    d = pos - p_ref
    d -= s["box"] * np.rint(d / s["box"])
    print(f"[two masses vs oracle] cfg={cfg} max |dx| {np.abs(d).max():.2e} "
          f"max |dv| {np.abs(v - v_ref).max():.2e}", flush=True)
    assert np.abs(d).max() < 1e-10, cfg
    assert np.abs(v - v_ref).max() < 1e-9, cfg
    assert P.force_error(f, f_ref) < 1e-9, cfg
    assert U == pytest.approx(ep[-1], rel=1e-10)


@pytest.mark.parametrize("prec", [0, 1])
def test_velocity_verlet_fused_step_with_early_rebuilds_bitwise(m, prec):
    # Fast particles cross skin/2 between scheduled rebuilds.  A staged force
    # call that takes the integrator step itself learns of the crossing only
    # after its launch; its records and velocities must then be dropped and
    # the step redone after the rebuild.  One call must still agree bit for
    # bit with one-step calls, which never fuse.
    import torch
    s = scenes.config1()
    v0 = 15.0 * s["vel"]
    cfg = (1, 2, 16, 4, 0, 0, 1)
    out = []
    for single in (False, True):
        with m.System(s["pos"], s["box"], s["rc"], skin=0.3, rebuild_every=6,
                      precision=prec) as sysm:
            sysm.set_config(cfg)
            vel = [torch.tensor(np.ascontiguousarray(v0[:, k]), device="cuda") for k in range(3)]
            sysm.set_timing(True)
            if single:
                for _ in range(24):
                    sysm.step_vv(vel, s["dt"], 1)
            else:
                sysm.step_vv(vel, s["dt"], 24)
            _, _, nf, nb = sysm.get_timing()
            out.append((sysm.get_positions(), torch.stack(vel, 1).cpu().numpy(), nb, nf))
    print(f"[fused step, early rebuilds] prec={prec} rebuilds {out[0][2]} / {out[1][2]}, "
          f"force calls {out[0][3]} / {out[1][3]}", flush=True)
    assert out[0][2] == out[1][2] >= 6, (out[0][2], out[1][2])  # the schedule alone gives 4
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])


def test_vl_fixed_point_frame_limits(m, orc):
    # The FP32-pair staged kernel reads fixed-point words of one frame per
    # box.  A long box at liquid density whose grid step is just under the
    # 1e-7 sigma limit (297 sigma) still meets the 1e-5 bar, with the cutoff
    # band derived from that step; at 323 sigma the step would exceed the
    # limit and the kernel is refused (MDLJ_ERR_ARG), while the all-FP64 one
    # is not.
    pos, box = scenes.fcc_lattice(170, 5, 5, 0.75, 0.05, seed=45)
    assert 0.9e-7 < P.fx_step(box, 2.5, 0.3) < 1e-7
    s = dict(pos=pos, box=box, rc=2.5, eps=[1.0], sig=[1.0], types=None)
    staged = [c for c in vl_configs(m) if len(c) == 7]
    check(m, orc, s, staged[:2] + staged[-2:], "297 sigma", precs=(0,), skin=0.3)
    pos, box = scenes.fcc_lattice(185, 5, 5, 0.75, 0.05, seed=46)
    assert P.fx_step(box, 2.5, 0.3) > 1e-7
    with m.System(pos, box, 2.5, skin=0.3, precision=0) as sysm:
        sysm.set_config(staged[0])
        with pytest.raises(m.MdljError) as ei:
            sysm.forces()
        assert ei.value.status == -1
        assert "fixed-point" in str(ei.value)
        sysm.set_precision(1)
        f, U, W = sysm.forces()
    ref = orc.forces(pos, box, 2.5)
    assert P.force_error(f, ref["f"]) <= 1e-12


def test_vl_cells_exactly_list_range_wide(m, orc):
    # box 16 x 1.75 = 28 = 10 x (rc + skin): cells exactly rc + skin wide, so
    # the list build may not drop candidates by cell halves
    pos, box = scenes.fcc_lattice(16, 16, 16, 4.0 / 1.75 ** 3, 0.05, seed=43)
    assert abs(box[0] - 28.0) < 1e-9
    s = dict(pos=pos, box=box, rc=2.5, eps=[1.0], sig=[1.0], types=None)
    cfgs = [(m.NBR_VL, m.ORD_WAVE_PER_I, 16, 4, 0, 0, 1), (m.NBR_VL, m.ORD_WAVE_PER_I, 8, 8, 0, 0),
            (m.NBR_VL, m.ORD_WAVE_PER_I, 8, 8, 0, 1), (m.NBR_VL, m.ORD_I_PER_LANE, 0, 0, 0, 0)]
    check(m, orc, s, cfgs, "edge=rl", skin=0.3)


def test_vl_rebuild_after_density_change_on_same_grid(m, orc):
    # the second build runs on the same grid with 25% denser cells on one
    # side, beyond the staging sizes remembered from the first build
    pos, box = scenes.fcc_lattice(14, 14, 14, 0.75, 0.05, seed=44)
    L = box[0]
    squeezed = pos.copy()
    x = squeezed[:, 0]
    left = x < 0.5 * L
    squeezed[left, 0] = 0.8 * x[left]
    squeezed[~left, 0] = 0.4 * L + 1.2 * (x[~left] - 0.5 * L)
    for cfg in ((m.NBR_VL, m.ORD_WAVE_PER_I, 16, 4, 0, 0, 1),
                (m.NBR_VL, m.ORD_WAVE_PER_I, 4, 16, 0, 1)):
        with m.System(pos, box, 2.5, skin=0.3, precision=1) as sysm:
            sysm.set_config(cfg)
            f, U, W = sysm.forces()
            ref = orc.forces(pos, box, 2.5)
            assert P.force_error(f, ref["f"]) <= 1e-12, cfg
            sysm.set_positions(squeezed)
            sysm.rebuild()
            f, U, W = sysm.forces()
            ref = orc.forces(squeezed, box, 2.5)
            assert P.force_error(f, ref["f"]) <= 1e-12, cfg
            assert U == pytest.approx(ref["U"], rel=1e-12), cfg
