"""The tuner on the GPU (section 2.3.2): its objective is the MD step as
mdlj_step_vv runs it, measured with time step 0, so tuning moves nothing
and does not count in the caller's kernel timing; the step time it reports
for its choice agrees with real velocity-Verlet steps; the early-stopping
search (section 6's cheaper tuning) lands within a few percent of the full
search with fewer samples."""
import time

import numpy as np
import pytest

from paper_2512_03565_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def m():
    from paper_2512_03565_amd import mdlj
    return mdlj


def test_tuning_moves_nothing_and_is_not_timed(m):
    s = scenes.config2()
    with m.System(s["pos"], s["box"], s["rc"], skin=0.3) as sysm:
        sysm.set_timing(True)
        sysm.forces()
        before = sysm.get_positions()
        sysm.tune(m.TUNE_EXHAUSTIVE, 2)
        after = sysm.get_positions()
        _, _, nf, nb = sysm.get_timing()
    assert np.array_equal(before, after)
    assert (nf, nb) == (1, 1)


def test_tuned_step_time_agrees_with_md_steps(m):
    import torch
    s = scenes.config2()
    n = len(s["pos"])
    v0 = scenes.mb_velocities(n, 1.0, 1.0, seed=91)
    with m.System(s["pos"], s["box"], s["rc"], skin=0.3, rebuild_every=10) as sysm:
        chosen, us = sysm.tune(m.TUNE_EXHAUSTIVE, 4)
        vel = [torch.tensor(np.ascontiguousarray(v0[:, k]), device="cuda") for k in range(3)]
        sysm.step_vv(vel, s["dt"], 20)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sysm.step_vv(vel, s["dt"], 200)
        torch.cuda.synchronize()
        md_us = (time.perf_counter() - t0) / 200 * 1e6
    print(f"[tuner] {m.config_name(chosen)}: tuned {us:.1f} us/step, MD {md_us:.1f} us/step",
          flush=True)
    assert 0.75 * md_us < us < 1.25 * md_us


@pytest.mark.parametrize("which", ["cfg2", 1601, 1613, 1650])
def test_early_stop_close_to_full_search_and_cheaper(m, which):
    s = scenes.config2() if which == "cfg2" else scenes.tuning_scene(which, n_max=4e5)
    types = s["types"] if len(s["eps"]) > 1 else None
    with m.System(s["pos"], s["box"], s["rc"], s["eps"], s["sig"], types=types, skin=0.3,
                  rebuild_every=10) as sysm:
        t0 = time.perf_counter()
        full_cfg, full_us = sysm.tune(m.TUNE_EXHAUSTIVE, 4)
        t_full = time.perf_counter() - t0
        table = sysm.tune_results()
        full_taken = sysm.tune_taken().sum()
        t0 = time.perf_counter()
        early_cfg, early_us = sysm.tune(m.TUNE_EARLY_STOP, 4)
        t_early = time.perf_counter() - t0
        early_taken = sysm.tune_taken().sum()
        # a second full search: how far two searches' tables differ
        sysm.tune(m.TUNE_EXHAUSTIVE, 4)
        table2 = sysm.tune_results()

        # both choices re-measured, interleaved, 10 samples each
        def timed(cfg):
            sysm.set_config(cfg)
            return sysm.tune(m.TUNE_FIXED, 10)[1]

        t_f = min(timed(full_cfg), timed(full_cfg))
        t_e = min(timed(early_cfg), timed(early_cfg))
    ok = np.isfinite(table) & np.isfinite(table2)
    spread = float(np.max(np.abs(table[ok] / table2[ok] - 1)))
    regret = t_e / t_f - 1
    print(f"[early stop] {which} n={len(s['pos'])}: full {m.config_name(full_cfg)} "
          f"({t_full:.2f} s, {full_taken} samples), early {m.config_name(early_cfg)} "
          f"({t_early:.2f} s, {early_taken} samples); re-measured {t_f:.1f} / {t_e:.1f} us, "
          f"regret {regret:.3f}; two full searches differ by up to {spread:.3f}", flush=True)
    assert early_taken < full_taken
    assert regret < 0.10
