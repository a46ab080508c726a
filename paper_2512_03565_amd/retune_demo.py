"""Workloads whose particle distribution changes, with runtime re-tuning
(the tuner's schedule of section 2.3.2: tune, run, check whether the scene
has changed, tune again; section 5 runs such scenes).

Workloads:
  droplet  a droplet of radius 40 at rho 0.8 in vapour at rho 0.05, 1M
           particles placed by Poisson-disk sampling (spacing 0.9), rc 3.0,
           T 0.9;
  explode  a dense block (1M particles, FCC at rho 0.75) released at
           T = 5 into a periodic box three times its size per axis, rc 2.5.
Skin 0.3, lists rebuilt every 10 steps (or earlier).  The run is cut into
blocks; before each block the eight scene features are read and compared
with those of the last tuning (`mdlj_retune_needed`: density or the spread
of cell occupancies moved by more than 10%), and the scene is tuned again
when they have.  Modes: fixed (linked cells, i-per-lane), exhaustive,
learned (the shipped network), early_stop.  Prints one JSON line per mode
with every block's features, trigger, configuration and ms/step.

    python -m paper_2512_03565_amd.retune_demo --workload droplet --steps 5000 --every 1000
"""
import argparse
import json
import os
import sys
import time

import numpy as np

WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "tuner_mlp.bin")
FEATURES = ["log10_n", "density", "rc_over_sigma", "species", "neighbours_rc", "occupancy_cv",
            "empty_cells", "max_over_mean"]


def make_scene(workload, n_total=1_000_000, r_drop=40.0):
    from paper_2512_03565_amd import scenes

    def progress(done, count):
        print(f"# scene: {done}/{count} points placed", file=sys.stderr, flush=True)

    if workload == "droplet":
        return scenes.config3(n_total=n_total, r_drop=r_drop, progress=progress)
    if workload == "explode":
        # about n_total particles: FCC cells 1 x 1 x 2 in proportion
        m = max(2, int(round((n_total / 8.0) ** (1.0 / 3.0))))
        return scenes.exploding_block(ncell=(m, m, 2 * m))
    raise ValueError(workload)


def run(mode, steps, every, samples, scene, seed=1013):
    import torch
    from paper_2512_03565_amd import mdlj, scenes
    s = scene
    n = len(s["pos"])
    vel0 = scenes.mb_velocities(n, s["T"], 1.0, seed=seed)
    stream = torch.cuda.current_stream()
    pos = torch.tensor(s["pos"], dtype=torch.float64, device="cuda")
    vel = [torch.tensor(np.ascontiguousarray(vel0[:, k]), device="cuda") for k in range(3)]
    blocks = []
    with mdlj.System(pos, s["box"], s["rc"], skin=s["skin"], rebuild_every=s["rebuild_every"],
                     stream=stream) as sysm:
        if mode in ("learned", "early_stop") and os.path.exists(WEIGHTS):
            sysm.mlp_load(WEIGHTS)
        kind = {"fixed": mdlj.TUNE_FIXED, "exhaustive": mdlj.TUNE_EXHAUSTIVE,
                "learned": mdlj.TUNE_LEARNED, "early_stop": mdlj.TUNE_EARLY_STOP}[mode]
        if mode == "fixed":
            sysm.set_config((mdlj.NBR_LC, mdlj.ORD_I_PER_LANE, 1, 1, 0, 0))
        feat_tuned = None
        tune_total = 0.0
        done = 0
        t_all = time.perf_counter()
        while done < steps:
            feat = sysm.features()
            retuned = False
            tune_s = 0.0
            if feat_tuned is None or (mode != "fixed" and mdlj.retune_needed(feat_tuned, feat)):
                t0 = time.perf_counter()
                sysm.tune(kind, samples)
                torch.cuda.synchronize()
                tune_s = time.perf_counter() - t0
                tune_total += tune_s
                feat_tuned = feat
                retuned = True
            k = min(every, steps - done)
            sysm.set_timing(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sysm.step_vv(vel, s["dt"], k)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            _, _, nf, nb = sysm.get_timing()
            sysm.set_timing(False)
            done += k
            b = {"first_step": done - k, "steps": k,
                 "config": mdlj.config_name(sysm.get_config()), "retuned": retuned,
                 "tuning_s": round(tune_s, 4), "ms_per_step": 1e3 * dt / k, "rebuilds": nb,
                 "features": {name: round(float(v), 5) for name, v in zip(FEATURES, feat)}}
            blocks.append(b)
            print(f"# {mode}: steps {done - k}..{done} {b['config']} {b['ms_per_step']:.3f} ms/step"
                  f"{' (retuned)' if retuned else ''} cv {feat[5]:.3f}", file=sys.stderr,
                  flush=True)
        wall = time.perf_counter() - t_all
        pairs = sysm.count_pairs()
    return {"mode": mode, "particles": n, "steps": steps, "useful_pairs_end": pairs,
            "wall_s": wall, "tuning_s": tune_total,
            "ms_per_step_incl_tuning": 1e3 * wall / steps,
            "retunes": int(sum(b["retuned"] for b in blocks)), "blocks": blocks}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=["droplet", "explode"], default="droplet")
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--every", type=int, default=1000)
    ap.add_argument("--samples", type=int, default=4)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--r-drop", type=float, default=40.0)
    ap.add_argument("--modes", default="fixed,exhaustive,learned,early_stop")
    a = ap.parse_args(argv)
    scene = make_scene(a.workload, a.n, a.r_drop)
    for mode in a.modes.split(","):
        r = run(mode, a.steps, a.every, a.samples, scene)
        r["workload"] = a.workload
        r["scene"] = scene["name"]
        print(json.dumps(r), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
