"""GPU tests of the pruned inner Verlet list of the staged kernels: the
entries closer than rc + 2 skin / 3 at the build (written by the list
build), read while no particle has moved more than skin / 3 since (the skin
argument of section 2.1.1 with the smaller skin), the full list
afterwards.  The inner list is off by default; these tests switch it on."""
import numpy as np
import pytest

from paper_2512_03565_amd import scenes
from tests import _parity as P

pytestmark = pytest.mark.gpu

STAGED = [(1, 2, 16, 4, 0, 0, 1), (1, 2, 8, 2, 0, 0, 1), (1, 2, 4, 8, 0, 0, 1)]


@pytest.fixture(scope="module")
def m():
    from paper_2512_03565_amd import mdlj
    return mdlj


@pytest.mark.parametrize("prec", [0, 1])
def test_inner_list_static_parity(m, orc, prec):
    s = scenes.config1()
    pos, box, rc = s["pos"], s["box"], s["rc"]
    ref = orc.forces(pos, box, rc)
    band = P.fx_band(box, rc, 0.3) if prec == 0 else P.F64_BAND
    slack, su, sw, _ = P.boundary_slack(orc, pos, box, rc, [1.0], [1.0], None, True, band)
    tol = 1e-5 if prec == 0 else 1e-12
    for cfg in STAGED:
        print(f"[prune] static prec={prec} cfg={cfg}", flush=True)
        with m.System(pos, box, rc, skin=0.3, precision=prec) as on, \
                m.System(pos, box, rc, skin=0.3, precision=prec) as off:
            on.set_config(cfg)
            on.set_pruning(True)
            off.set_config(cfg)
            assert on.pruning_state() == 0
            f0, _, _ = on.forces(energy=False)
            assert on.pruning_state() == 1
            f1, U1, W1 = on.forces()
            assert on.pruning_state() == 1
            assert np.array_equal(f0, on.forces(energy=False)[0])
            g, Ug, Wg = off.forces()
            assert off.pruning_state() == 0
            # the inner list drops only pairs beyond the cutoff: the same
            # pair terms, summed in another order
            assert np.abs(f1 - g).max() <= 1e-12 * P.frms(g) * 10, cfg
            assert P.force_error(f1, ref["f"], slack) <= tol
            assert P.total_error(U1, ref["U"], su) <= tol
            assert P.total_error(W1, ref["W"], sw) <= tol
            assert U1 == pytest.approx(Ug, rel=1e-12) and W1 == pytest.approx(Wg, rel=1e-12)


def _pair_scene():
    # a simple cubic gas at spacing 4 (no pair within rc + skin) in which
    # particle B sits 0.01 beyond r_in = rc + 0.2 from particle A along x:
    # the pair is in the full list but not in the inner one
    k = 6
    g = np.stack(np.meshgrid(*(np.arange(k) * 4.0 + 1.0,) * 3, indexing="ij"), -1).reshape(-1, 3)
    box = np.full(3, 4.0 * k)
    ia = 0                                  # site (0, 0, 0)
    ib = k * k                              # site (1, 0, 0)
    g[ib] = g[ia] + np.array([2.5 + 0.2 + 0.01, 0.0, 0.0])
    return g, box, ia, ib


@pytest.mark.parametrize("prec", [0, 1])
def test_inner_list_invalidated_by_displacement(m, orc, prec):
    pos, box, ia, ib = _pair_scene()
    rc = 2.5
    tol = 1e-5 if prec == 0 else 1e-12
    with m.System(pos, box, rc, skin=0.3, rebuild_every=1000, precision=prec) as sysm:
        sysm.set_config(STAGED[0])
        sysm.set_pruning(True)
        f, _, _ = sysm.forces()
        assert sysm.pruning_state() == 1 and np.abs(f).max() == 0.0
        # each of A, B 0.09 towards the other (< skin / 3 = 0.1): still
        # beyond rc, inner list valid
        p = pos.copy()
        p[ia, 0] += 0.09
        p[ib, 0] -= 0.09
        sysm.set_positions(p)
        f, _, _ = sysm.forces()
        assert sysm.pruning_state() == 1 and np.abs(f).max() == 0.0
        # 0.11 each (> skin / 3, < skin / 2): the pair is now inside rc and
        # absent from the inner list, which must be given up for the full one
        p = pos.copy()
        p[ia, 0] += 0.11
        p[ib, 0] -= 0.11
        sysm.set_positions(p)
        f, U, W = sysm.forces()
        # the tiles around A and B gave the inner list up, the others kept it
        state, tiles = sysm.pruning_state(tiles=True)
        assert state == 2 and 1 <= tiles <= 54, (state, tiles)
        ref = orc.forces(p, box, rc)
        assert np.abs(ref["f"][ia]).max() > 0.01
        err = np.abs(f - ref["f"]).max() / np.abs(ref["f"]).max()
        print(f"[prune] invalidation prec={prec} err {err:.3e}", flush=True)
        assert err <= tol
        # back within the bound: the word stays set until the next build
        sysm.set_positions(pos)
        sysm.forces()
        assert sysm.pruning_state(tiles=True) == (state, tiles)
        # every particle moved past the bound (0.07 per axis, 0.12 < skin / 2):
        # no tile keeps it
        sysm.set_positions(pos + 0.07)
        sysm.forces()
        assert sysm.pruning_state() == 3
        sysm.rebuild()
        assert sysm.pruning_state() == 1
        sysm.forces()
        assert sysm.pruning_state() == 1


@pytest.mark.parametrize("prec", [0, 1])
def test_inner_list_invalidated_inside_the_fused_step(m, orc, prec):
    # A and B approach at speed 1 each (dt 0.01): after step 10 each has
    # moved 0.1 (the bound), after 11 they are inside rc.  The integrator
    # steps inside the staged kernel must give the inner list up in time in
    # the tiles around them: the trajectory matches the oracle's
    import torch
    pos, box, ia, ib = _pair_scene()
    rc, dt, nsteps = 2.5, 0.01, 14
    vel = np.zeros_like(pos)
    vel[ia, 0] = 1.0
    vel[ib, 0] = -1.0
    p_ref, v_ref, f_ref, ep, _ = orc.vv(pos, vel, box, rc, dt, nsteps)
    assert np.abs(f_ref[ia]).max() > 0.01
    with m.System(pos, box, rc, skin=0.3, rebuild_every=1000, precision=prec) as sysm:
        sysm.set_config(STAGED[0])
        sysm.set_pruning(True)
        sysm.set_timing(True)
        v = [torch.tensor(np.ascontiguousarray(vel[:, k]), device="cuda") for k in range(3)]
        sysm.step_vv(v, dt, nsteps)
        _, _, nf, nb = sysm.get_timing()
        # the tiles around A and B gave the inner list up, the others kept it
        state, tiles = sysm.pruning_state(tiles=True)
        assert state == 2 and 1 <= tiles <= 54, (state, tiles)
        pos_g = sysm.get_positions()
    assert nb == 1, nb   # one build: skin / 2 is never crossed
    vg = torch.stack(v, 1).cpu().numpy()
    d = pos_g - p_ref
    d -= box * np.rint(d / box)
    tol = 1e-6 if prec == 0 else 1e-10
    print(f"[prune] fused prec={prec} dx {np.abs(d).max():.3e} dv {np.abs(vg - v_ref).max():.3e}",
          flush=True)
    assert np.abs(d).max() < tol
    assert np.abs(vg - v_ref).max() < 100 * tol


def test_inner_list_vv_matches_unpruned(m):
    # config 1 dynamics over two list periods: pruned and unpruned runs
    # agree to the order of the FP64 sums
    import torch
    s = scenes.config1()
    out = []
    for prune in (True, False):
        with m.System(s["pos"], s["box"], s["rc"], skin=0.3, rebuild_every=10,
                      precision=1) as sysm:
            sysm.set_config(STAGED[0])
            sysm.set_pruning(prune)
            v = [torch.tensor(np.ascontiguousarray(s["vel"][:, k]), device="cuda")
                 for k in range(3)]
            sysm.step_vv(v, s["dt"], 20)
            out.append((sysm.get_positions(), torch.stack(v, 1).cpu().numpy()))
    d = out[0][0] - out[1][0]
    d -= s["box"] * np.rint(d / s["box"])
    print(f"[prune] vv pruned vs unpruned dx {np.abs(d).max():.3e}", flush=True)
    assert np.abs(d).max() < 1e-11
    assert np.abs(out[0][1] - out[1][1]).max() < 1e-9


def test_pruning_argument_checks(m):
    s = scenes.config1()
    with m.System(s["pos"], s["box"], s["rc"], skin=0.3) as sysm:
        with pytest.raises(m.MdljError):
            m.check(m.lib.mdlj_set_pruning(sysm.ctx, 2), sysm.ctx)
        sysm.set_config(STAGED[0])
        sysm.forces()
        assert sysm.pruning_state() == 0  # off by default
        sysm.set_pruning(True)
        sysm.forces()
        assert sysm.pruning_state() == 1
        # switching it off drops the inner list at once
        sysm.set_pruning(False)
        assert sysm.pruning_state() == 0
        sysm.forces()
        assert sysm.pruning_state() == 0
    # no skin: no inner list
    with m.System(s["pos"], s["box"], s["rc"], skin=0.0) as sysm:
        sysm.set_config(STAGED[0])
        sysm.set_pruning(True)
        sysm.forces()
        assert sysm.pruning_state() == 0
