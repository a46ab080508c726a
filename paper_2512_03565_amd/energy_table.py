"""Energy against time as the tuning metric (section 2.3.3; section 5's
Benchmark B compares the two optima).

For one scene, the full search runs twice over every configuration: once
by time per MD step (4 cycles of rebuild-interval steps, the first dropped)
and once by energy per MD step (mean board power over --windows refreshes
of the GPU's energy counter, about a second each, times the step time of
the same run).  Prints one JSON line per configuration and a summary line
naming both optima.

    python -m paper_2512_03565_amd.energy_table --scene 1M --windows 2
"""
import argparse
import json
import sys

import numpy as np


def run(scene, windows):
    import torch
    from paper_2512_03565_amd import mdlj, scenes
    s = scenes.headline() if scene == "1M" else scenes.config2()
    pos = torch.tensor(s["pos"], dtype=torch.float64, device="cuda")
    with mdlj.System(pos, s["box"], s["rc"], skin=s["skin"], rebuild_every=s["rebuild_every"],
                     stream=torch.cuda.current_stream()) as sysm:
        names = [mdlj.config_name(c) for c in sysm.configs()]
        sysm.set_tune_metric(mdlj.METRIC_TIME)
        t_cfg, _ = sysm.tune(mdlj.TUNE_EXHAUSTIVE, 4)
        us = sysm.tune_results()
        sysm.set_tune_metric(mdlj.METRIC_ENERGY)
        e_cfg, _ = sysm.tune(mdlj.TUNE_EXHAUSTIVE, windows)
        uj = sysm.tune_results()
        watts = sysm.tune_power()
    for k, name in enumerate(names):
        print(json.dumps({"table": "energy", "scene": scene, "config": name,
                          "us_per_step": None if not np.isfinite(us[k]) else float(us[k]),
                          "uj_per_step": None if not np.isfinite(uj[k]) else float(uj[k]),
                          "watts": None if not np.isfinite(watts[k]) else float(watts[k])}),
              flush=True)
    tn, en = mdlj.config_name(t_cfg), mdlj.config_name(e_cfg)
    kt, ke = names.index(tn), names.index(en)
    print(json.dumps({"table": "energy_summary", "scene": scene, "time_optimum": tn,
                      "energy_optimum": en, "differ": tn != en,
                      "energy_of_time_optimum_uj": float(uj[kt]),
                      "energy_of_energy_optimum_uj": float(uj[ke]),
                      "time_of_time_optimum_us": float(us[kt]),
                      "time_of_energy_optimum_us": float(us[ke])}), flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--scene", choices=["100k", "1M"], default="1M")
    ap.add_argument("--windows", type=int, default=2)
    a = ap.parse_args(argv)
    run(a.scene, a.windows)
    return 0


if __name__ == "__main__":
    sys.exit(main())
