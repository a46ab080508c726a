"""Timing tables beside the benchmark.

orders: the 100,000-particle FCC scene (rho 0.75, rc 2.5, skin 0.3, lists
rebuilt every 10 steps), or with --scene 1M the 1,000,000-particle headline
scene, in FP32 pair arithmetic (or --prec f64): every configuration of the
search space runs --steps velocity-Verlet steps; ms per step, force-kernel
and rebuild times from the library's events.

precision: the 4,000,000-particle two-species scene (rho 0.7, rc 3.0,
Lorentz-Berthelot): Verlet cluster lists with clusters of 4 and 8, FP32 pair
arithmetic with FP64 accumulation against the all-FP64 kernels; force-kernel
time over --reps evaluations.

sizes: the headline's scene (FCC at rho 0.75, rc 2.5, skin 0.3, T 1.0)
from 32k to 16M particles on one GPU, each tuned by the full search and
then run for --steps velocity-Verlet steps: what one GPU's share of a
larger system costs at each size.

Prints one JSON line per row.

    python -m paper_2512_03565_amd.orders_table orders --steps 200
    python -m paper_2512_03565_amd.orders_table precision --reps 20
    python -m paper_2512_03565_amd.orders_table sizes --steps 100
"""
import argparse
import json
import sys
import time

import numpy as np


def orders(steps, scene="100k", prec="f32"):
    import torch
    from paper_2512_03565_amd import mdlj, scenes
    s = scenes.config2() if scene == "100k" else scenes.headline()
    workload = ("100k FCC rho0.75 rc2.5 skin0.3" if scene == "100k"
                else "1M FCC 50x50x100 rho0.75 rc2.5 skin0.3")
    n = len(s["pos"])
    vel0 = scenes.mb_velocities(n, s["T"], 1.0, seed=1012)
    pos = torch.tensor(s["pos"], dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    with mdlj.System(pos, s["box"], s["rc"], skin=s["skin"], rebuild_every=s["rebuild_every"],
                     stream=stream,
                     precision=mdlj.PREC_F64 if prec == "f64" else mdlj.PREC_F32PAIR_F64ACC) as sysm:
        pairs = sysm.count_pairs()
        for cfg in sysm.configs():
            sysm.set_positions(pos)
            sysm.set_config(cfg)
            vel = [torch.tensor(np.ascontiguousarray(vel0[:, k]), device="cuda") for k in range(3)]
            sysm.step_vv(vel, s["dt"], 10)
            torch.cuda.synchronize()
            sysm.set_timing(True)
            t0 = time.perf_counter()
            sysm.step_vv(vel, s["dt"], steps)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            f_us, b_us, nf, nb = sysm.get_timing()
            sysm.set_timing(False)
            print(json.dumps({"table": "orders", "workload": workload, "precision": prec,
                              "config": mdlj.config_name(cfg), "steps": steps,
                              "ms_per_step": 1e3 * wall / steps,
                              "mpairs_per_s": pairs * steps / wall / 1e6,
                              "force_us": f_us / max(nf, 1),
                              "rebuild_us": b_us / max(nb, 1), "rebuilds": nb}), flush=True)


def precision(reps):
    import torch
    from paper_2512_03565_amd import mdlj, scenes
    s = scenes.config4()
    pos = torch.tensor(s["pos"], dtype=torch.float64, device="cuda")
    types = torch.tensor(s["types"], dtype=torch.int32, device="cuda")
    n = len(s["pos"])
    out = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(3)]
    stream = torch.cuda.current_stream()
    names = ["VCL4/cluster-tile/4x16", "VCL4/i-per-lane", "VCL8/cluster-tile/8x8",
             "VCL8/i-per-lane", "VCL4/cluster-tile/4x16/n3", "VL/wave-per-i/16x4",
             "VL/wave-per-i/16x4/lds"]
    with mdlj.System(pos, s["box"], s["rc"], s["eps"], s["sig"], types=types, skin=s["skin"],
                     rebuild_every=1000, stream=stream) as sysm:
        pairs = sysm.count_pairs()
        space = {mdlj.config_name(c): c for c in sysm.configs()}
        for name in names:
            for prec in (mdlj.PREC_F32PAIR_F64ACC, mdlj.PREC_F64):
                sysm.set_precision(prec)
                try:
                    sysm.set_config(space[name])
                    sysm.forces(out=out, energy=False)
                except mdlj.MdljError as e:
                    print(json.dumps({"table": "precision", "config": name, "error": str(e)}),
                          flush=True)
                    break
                sysm.set_timing(True)
                for _ in range(reps):
                    sysm.forces(out=out, energy=False)
                f_us, _, nf, _ = sysm.get_timing()
                sysm.set_timing(False)
                us = f_us / max(nf, 1)
                print(json.dumps({"table": "precision",
                                  "workload": "4M two-species FCC rho0.7 rc3.0",
                                  "config": name, "precision": "f32pair" if prec == 0 else "f64",
                                  "force_us": us, "mpairs_per_s": pairs / us}), flush=True)


# the largest as a cube: its box (280 sigma) stays inside the FP32 staged
# kernel's fixed-point frame, which a 220 x 220 x 440 box of the same
# count would leave
SIZES = [(16, 16, 32), (32, 32, 64), (50, 50, 100), (80, 80, 160), (160, 160, 160)]


def sizes(steps):
    import torch
    from paper_2512_03565_amd import mdlj, scenes
    for nc in SIZES:
        pos_h, box = scenes.fcc_lattice(nc[0], nc[1], nc[2], 0.75, 0.05, 1013)
        n = len(pos_h)
        vel0 = scenes.mb_velocities(n, 1.0, 1.0, seed=1014)
        pos = torch.tensor(pos_h, dtype=torch.float64, device="cuda")
        del pos_h
        with mdlj.System(pos, box, 2.5, skin=0.3, rebuild_every=10,
                         stream=torch.cuda.current_stream()) as sysm:
            pairs = sysm.count_pairs()
            t0 = time.perf_counter()
            cfg, tuned_us = sysm.tune(mdlj.TUNE_EXHAUSTIVE, 4)
            tune_s = time.perf_counter() - t0
            vel = [torch.tensor(np.ascontiguousarray(vel0[:, k]), device="cuda") for k in range(3)]
            sysm.step_vv(vel, 0.002, 10)
            torch.cuda.synchronize()
            sysm.set_timing(True)
            t0 = time.perf_counter()
            sysm.step_vv(vel, 0.002, steps)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            f_us, b_us, nf, nb = sysm.get_timing()
            fused_us, nfused = sysm.get_timing_fused()
            sysm.set_timing(False)
        print(json.dumps({"table": "sizes", "fcc_cells": list(nc), "particles": n,
                          "useful_pairs": pairs, "config": mdlj.config_name(cfg),
                          "tuning_s": tune_s, "steps": steps, "ms_per_step": 1e3 * wall / steps,
                          "mpairs_per_s": pairs * steps / wall / 1e6,
                          "ns_per_particle_step": 1e9 * wall / steps / n,
                          "force_us": f_us / max(nf, 1),
                          "fused_us": fused_us / nfused if nfused else None,
                          "rebuild_us": b_us / max(nb, 1)}), flush=True)
        del pos, vel, sysm
        torch.cuda.empty_cache()


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("table", choices=["orders", "precision", "sizes"])
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--scene", choices=["100k", "1M"], default="100k")
    ap.add_argument("--prec", choices=["f32", "f64"], default="f32")
    a = ap.parse_args(argv)
    if a.table == "orders":
        orders(a.steps, a.scene, a.prec)
    elif a.table == "precision":
        precision(a.reps)
    else:
        sizes(a.steps)
    return 0


if __name__ == "__main__":
    sys.exit(main())
