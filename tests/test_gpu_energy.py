"""Energy as the tuning metric on the GPU (section 2.3.3): the energy
counter read through AMD SMI advances, and a configuration's measured
energy per step is its mean power times its step time, with power in the
range a busy MI355X board draws and slower configurations costing more
energy per step at similar power."""
import numpy as np
import pytest

from paper_2512_03565_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def m():
    from paper_2512_03565_amd import mdlj
    return mdlj


def test_energy_counter_and_per_step_energy(m):
    s = scenes.config2()
    with m.System(s["pos"], s["box"], s["rc"], skin=0.3, rebuild_every=10) as sysm:
        j0, t0 = sysm.gpu_energy()
        names = [m.config_name(c) for c in sysm.configs()]
        rows = {}
        for name in ("VL/wave-per-i/16x4/lds", "LC/i-per-lane/k1"):
            sysm.set_config(sysm.configs()[names.index(name)])
            sysm.set_tune_metric(m.METRIC_TIME)
            _, us = sysm.tune(m.TUNE_FIXED, 4)
            sysm.set_tune_metric(m.METRIC_ENERGY)
            _, uj = sysm.tune(m.TUNE_FIXED, 2)
            rows[name] = (us, uj)
            print(f"[energy] {name}: {us:.1f} us/step, {uj:.0f} uJ/step, "
                  f"{uj / us:.0f} W", flush=True)
        j1, t1 = sysm.gpu_energy()
        with pytest.raises(m.MdljError):
            sysm.tune(m.TUNE_EARLY_STOP, 4)
    assert j1 > j0 and t1 > t0
    for name, (us, uj) in rows.items():
        w = uj / us
        assert 100.0 < w < 2000.0, (name, w)
    fast, slow = rows["VL/wave-per-i/16x4/lds"], rows["LC/i-per-lane/k1"]
    assert slow[1] > 2.0 * fast[1]
