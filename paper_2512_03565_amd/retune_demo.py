"""Droplet workload with runtime re-tuning (the tuner's schedule of
section 2.3.2: tune, run, check whether the scene has changed, tune again).

A spherical droplet (radius 40, rho 0.8) in vapour (rho 0.05), about 1M
particles, rc 3.0, T 0.9, Verlet skin 0.3 rebuilt every 10 steps.  The run
is cut into blocks; before each block the eight scene features are read and
compared with those of the last tuning (`mdlj_retune_needed`: density or
the spread of cell occupancies moved by more than 10%); the scene is tuned
again when they have.  Modes: fixed (linked cells, i-per-lane), exhaustive, learned
(with the shipped network).  Prints one JSON line per mode.

    python -m paper_2512_03565_amd.retune_demo --steps 5000 --every 1000
"""
import argparse
import json
import os
import sys
import time

import numpy as np

WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "tuner_mlp.bin")


def run(mode, steps, every, samples, n_total, r_drop=40.0):
    import torch
    from paper_2512_03565_amd import mdlj, scenes
    s = scenes.config3(n_total=n_total, r_drop=r_drop)
    n = len(s["pos"])
    vel0 = scenes.mb_velocities(n, s["T"], 1.0, seed=1013)
    stream = torch.cuda.current_stream()
    pos = torch.tensor(s["pos"], dtype=torch.float64, device="cuda")
    vel = [torch.tensor(np.ascontiguousarray(vel0[:, k]), device="cuda") for k in range(3)]
    blocks = []
    with mdlj.System(pos, s["box"], s["rc"], skin=s["skin"], rebuild_every=s["rebuild_every"],
                     stream=stream) as sysm:
        if mode == "learned" and os.path.exists(WEIGHTS):
            sysm.mlp_load(WEIGHTS)
        kind = {"fixed": mdlj.TUNE_FIXED, "exhaustive": mdlj.TUNE_EXHAUSTIVE,
                "learned": mdlj.TUNE_LEARNED}[mode]
        if mode == "fixed":
            sysm.set_config((mdlj.NBR_LC, mdlj.ORD_I_PER_LANE, 1, 1, 0, 0))
        feat_tuned = None
        tune_total = 0.0
        done = 0
        t_all = time.perf_counter()
        while done < steps:
            feat = sysm.features()
            retuned = False
            if feat_tuned is None or (mode != "fixed" and mdlj.retune_needed(feat_tuned, feat)):
                t0 = time.perf_counter()
                sysm.tune(kind, samples)
                torch.cuda.synchronize()
                tune_total += time.perf_counter() - t0
                feat_tuned = feat
                retuned = True
            k = min(every, steps - done)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sysm.step_vv(vel, s["dt"], k)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            done += k
            blocks.append({"steps": k, "config": mdlj.config_name(sysm.get_config()),
                           "retuned": retuned, "ms_per_step": 1e3 * dt / k,
                           "density": float(feat[1]), "occupancy_cv": float(feat[5])})
        wall = time.perf_counter() - t_all
        pairs = sysm.count_pairs()
    return {"mode": mode, "particles": n, "steps": steps, "useful_pairs_end": pairs,
            "wall_s": wall, "tuning_s": tune_total,
            "ms_per_step_incl_tuning": 1e3 * wall / steps,
            "retunes": int(sum(b["retuned"] for b in blocks)), "blocks": blocks}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--every", type=int, default=1000)
    ap.add_argument("--samples", type=int, default=10)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--r-drop", type=float, default=40.0)
    ap.add_argument("--modes", default="fixed,exhaustive,learned")
    a = ap.parse_args(argv)
    for mode in a.modes.split(","):
        print(json.dumps(run(mode, a.steps, a.every, a.samples, a.n, a.r_drop)), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
