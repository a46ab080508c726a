"""Benchmark: LJ 12-6 molecular dynamics steps on one MI355X.

Workload (synthetic, generated from a seed): 1,000,000 single-species LJ
particles on a 50x50x100 FCC lattice at density 0.75 (box 87.358 x 87.358 x
174.716 sigma, periodic), jittered by +-0.05 sigma, Maxwell-Boltzmann
velocities at T = 1.0, cutoff 2.5 sigma, Verlet skin 0.3 sigma, lists
rebuilt every 10 steps, dt = 0.002, FP32 pair arithmetic with FP64
accumulation.

A step is one velocity-Verlet MD step through the library: half kick and
drift, neighbour upkeep (re-binning for linked cells; displacement check and
record refresh, or a rebuild every 10th step, for lists), the force kernel
of the chosen configuration (forces only), un-permute, half kick.  With
staged Verlet lists the force kernel itself takes the kicks, the drift and
the displacement test between rebuilds; the roofline line then describes
that kernel (its time from the events around those launches).

Before the timed region the configuration is chosen four ways: fixed
(linked cells, i-per-lane -- the one-order baseline), exhaustive full search,
the learned tuner and the early-stopping search; each is then run for
--steps steps.  A fifth mode runs the full search's choice in all-FP64
arithmetic.  The tuners score configurations by the MD step itself.  The
headline value is the exhaustive choice's throughput in useful pairs
(r < rc, unordered) per second.

Prints one JSON line.  --gpus > 1 is refused: the library runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Useful FLOPs per unordered pair in the canonical Newton-3 form (FMA = 2,
# reciprocal = 1): separation 3, r^2 5, 1/r^2 1, s2 1, s6 2, force factor 5,
# scaling 3, +F_i 3, -F_j 3 = 26 for forces; energy and virial add 7 (33).
# MD steps here compute forces only.
FLOP_PER_PAIR = 26.0
PEAK_FP32 = 157.3e12     # MI355X vector FP32 (packed) FLOP/s
PEAK_HBM = 8.0e12        # MI355X HBM3E bytes/s
TUNER_WEIGHTS = os.path.join(ROOT, "paper_2512_03565_amd", "data", "tuner_mlp.bin")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--samples", type=int, default=4,
                    help="tuning samples (cycles of rebuild-interval MD steps) per configuration")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="budget of the oracle CPU baseline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--only", default=None,
                    help="run one mode only: fixed|exhaustive|learned|early_stop|fp64")
    ap.add_argument("--config", default=None,
                    help="run this configuration (by name) without tuning, e.g. for profiling")
    ap.add_argument("--prune", action="store_true",
                    help="switch the pruned inner Verlet list on (for comparison)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="afterwards, copy a MIB-MiB device buffer 5 times (a plain copy of "
                         "known size, to scale hardware byte counters)")
    return ap.parse_args()


def run_mode(m, torch, sysm, vel, dt, steps, warmup, pairs):
    """Warm up, then time `steps` MD steps; returns dict of measurements."""
    if warmup:
        sysm.step_vv(vel, dt, warmup)
    torch.cuda.synchronize()
    sysm.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sysm.step_vv(vel, dt, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    force_us, build_us, nf, nb = sysm.get_timing()
    fused_us, nfused = sysm.get_timing_fused()
    sysm.set_timing(False)
    ms_step = 1e3 * wall / steps
    kern_us = force_us / max(nf, 1)
    return {
        "ms_per_step": ms_step,
        "mpairs_per_s": pairs * steps / wall / 1e6,
        "force_kernel_us": kern_us,
        "force_kernel_mpairs_per_s": pairs / kern_us,
        # force kernels that also took the integrator step (staged lists)
        "fused_kernel_us": fused_us / nfused if nfused else None,
        "fused_calls": nfused,
        "force_calls": nf,
        "rebuild_us": build_us / max(nb, 1),
        "rebuilds": nb,
    }


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "vl_lds_16x4_headline_1M_traffic.json")


def measured_traffic(config_name, fused):
    """HBM bytes per launch of the force kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE, scaled by what the same counters read
    for a copy of known size); None unless it was taken for this
    configuration and the kernel sources are unchanged since."""
    import hashlib
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except OSError:
        return None
    if t.get("config") != config_name or bool(t.get("fused")) != fused:
        return None
    h = hashlib.sha256()
    for rel in t["source_files"]:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return t["traffic_bytes_per_launch"] if h.hexdigest() == t["source_sha256"] else None


def rooflines(flops, kernel_us, list_bytes):
    """The dominant kernel against both ceilings: its useful FLOPs over the
    FP32 vector peak and, with Verlet lists, its algorithmic bytes over HBM
    bandwidth.  The roofline that bounds it is the ceiling that alone takes
    longer for its work (the lower attainable rate at its arithmetic
    intensity); returns (bounding, other), other None without lists."""
    t = kernel_us * 1e-6
    alu = {"bound": "alu", "achieved": flops / t / 1e12, "peak": PEAK_FP32 / 1e12,
           "unit": "TFLOP/s", "frac": flops / t / PEAK_FP32, "flop_per_pair": FLOP_PER_PAIR}
    if not list_bytes:
        return alu, None
    hbm = {"bound": "hbm", "achieved": list_bytes / t / 1e9, "peak": PEAK_HBM / 1e9,
           "unit": "GB/s", "frac": list_bytes / t / PEAK_HBM, "algorithmic_bytes": list_bytes,
           "flop_per_byte": flops / list_bytes}
    if list_bytes / PEAK_HBM > flops / PEAK_FP32:
        return hbm, alu
    return alu, hbm


def list_stream_bytes(sysm, n, fused):
    """Algorithmic bytes of one launch of the FP32-pair staged Verlet-list
    kernel: the stored list entries (rows padded to 8), the list lengths
    (4 B per particle), the fixed-point x, y, z words of every sorted record
    once (12 B), and either the forces written (24 B per particle) or, when
    the launch takes the integrator step, that step's bytes per particle:
    record read and written (32 + 32), velocity read and written (24 + 24),
    list-build reference read (24), new words written (12).  None when the
    structure holds no Verlet lists."""
    entries, esize, records = sysm.neighbor_stats()
    if entries == 0:
        return None
    return entries * esize + 4 * n + 12 * records + (148 if fused else 24) * n


def cpu_model():
    """The host CPU's model name (Linux), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def physical_cores():
    """Physical cores among the CPUs this process may run on (Linux), or None."""
    try:
        allowed = os.sched_getaffinity(0)
        cores = set()
        cpu = phys = core = None
        with open("/proc/cpuinfo") as f:
            for line in f:
                k, _, v = line.partition(":")
                k = k.strip()
                if k == "processor":
                    cpu = int(v)
                elif k == "physical id":
                    phys = int(v)
                elif k == "core id":
                    core = int(v)
                elif not k and cpu is not None:
                    if cpu in allowed:
                        cores.add((phys, core))
                    cpu = phys = core = None
        if cpu is not None and cpu in allowed:
            cores.add((phys, core))
        return len(cores) or None
    except (OSError, ValueError):
        return None


def oracle_threads():
    return int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0)) or 1))


def cpu_baseline(scene, budget_s):
    import oracle
    nthreads = oracle_threads()
    t_total = 0.0
    reps = 0
    while t_total < budget_s and reps < 20:
        t0 = time.perf_counter()
        oracle.forces(scene["pos"], scene["box"], scene["rc"], nthreads=nthreads)
        t_total += time.perf_counter() - t0
        reps += 1
    return t_total / reps, reps, nthreads


def other_oracle_timings(nth):
    """The oracle on the 100k scene (full evaluation) and on a seeded
    50,000-particle sample of the 4M two-species scene (forces on the sample
    only), with the GPU-side pair counts they cover."""
    import oracle
    from paper_2512_03565_amd import scenes
    out = {}
    s = scenes.config2()
    t0 = time.perf_counter()
    oracle.forces(s["pos"], s["box"], s["rc"], nthreads=nth)
    t = time.perf_counter() - t0
    pi, _, _ = oracle.pairs_within(s["pos"], s["box"], s["rc"])
    out["100k_fcc_rho0.75"] = {"ms_per_eval": 1e3 * t, "mpairs_per_s": len(pi) / t / 1e6,
                               "threads": nth}
    s = scenes.config4()
    idx = np.sort(np.random.default_rng(20251205).choice(len(s["pos"]), 50_000, replace=False))
    t0 = time.perf_counter()
    oracle.forces_subset(s["pos"], s["box"], s["rc"], idx, s["eps"], s["sig"], s["types"],
                         nthreads=nth)
    t = time.perf_counter() - t0
    out["4M_two_species_50k_sample"] = {"ms_per_eval": 1e3 * t,
                                        "particles_per_s": len(idx) / t, "threads": nth}
    return out


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(a spatial decomposition into one brick per GPU, with halo exchange, "
              "is how the work would shard)", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs the GPU"
    torch.cuda.set_device(0)
    from paper_2512_03565_amd import mdlj, scenes

    s = scenes.headline()
    n = len(s["pos"])
    vel0 = scenes.mb_velocities(n, s["T"], 1.0, seed=20251204)
    stream = torch.cuda.current_stream()
    pos_d = torch.tensor(s["pos"], dtype=torch.float64, device="cuda")
    sysm = mdlj.System(pos_d, s["box"], s["rc"], skin=s["skin"], rebuild_every=s["rebuild_every"],
                       precision=mdlj.PREC_F32PAIR_F64ACC, stream=stream)
    if args.prune:
        sysm.set_pruning(True)
    pairs = sysm.count_pairs()
    results = {}
    modes = ["fixed", "exhaustive", "learned", "early_stop", "fp64"]
    if args.only:
        modes = [args.only]
    if args.config:
        modes = ["given"]
    for mode in modes:
        sysm.set_precision(mdlj.PREC_F64 if mode == "fp64" else mdlj.PREC_F32PAIR_F64ACC)
        sysm.set_positions(pos_d)
        vel = [torch.tensor(np.ascontiguousarray(vel0[:, k]), device="cuda") for k in range(3)]
        t0 = time.perf_counter()
        if mode == "given":
            names = [mdlj.config_name(c) for c in sysm.configs()]
            if args.config not in names:
                sys.exit(f"unknown configuration {args.config!r}; one of {names}")
            sysm.set_config(sysm.configs()[names.index(args.config)])
            cfg, tune_us = sysm.tune(mdlj.TUNE_FIXED, args.samples)
        elif mode == "fixed":
            sysm.set_config((mdlj.NBR_LC, mdlj.ORD_I_PER_LANE, 1, 1, 0, 0))
            cfg, tune_us = sysm.tune(mdlj.TUNE_FIXED, args.samples)
        elif mode == "exhaustive":
            cfg, tune_us = sysm.tune(mdlj.TUNE_EXHAUSTIVE, args.samples)
            table = sysm.tune_results()
            space = [mdlj.config_name(c) for c in sysm.configs()]
        elif mode == "fp64":
            cfg, tune_us = sysm.tune(mdlj.TUNE_EXHAUSTIVE, args.samples)
        elif mode == "early_stop":
            if os.path.exists(TUNER_WEIGHTS):
                sysm.mlp_load(TUNER_WEIGHTS)
            cfg, tune_us = sysm.tune(mdlj.TUNE_EARLY_STOP, args.samples)
        else:
            if os.path.exists(TUNER_WEIGHTS):
                sysm.mlp_load(TUNER_WEIGHTS)
            cfg, tune_us = sysm.tune(mdlj.TUNE_LEARNED, args.samples)
        tune_s = time.perf_counter() - t0
        r = run_mode(mdlj, torch, sysm, vel, s["dt"], args.steps, args.warmup, pairs)
        r["config"] = mdlj.config_name(cfg)
        fused = r["fused_kernel_us"] is not None
        sb = list_stream_bytes(sysm, n, fused)
        if sb is not None:
            r["list_stream_bytes"] = sb
            t_us = r["fused_kernel_us"] if fused else r["force_kernel_us"]
            r["list_stream_GBps"] = sb / (t_us * 1e-6) / 1e9
        r["tuned_step_us"] = tune_us
        r["tuning_s"] = tune_s
        if mode in ("exhaustive", "early_stop", "fp64"):
            r["tuning_samples"] = int(sysm.tune_taken().sum())
        if mode == "fp64":
            r["precision"] = "all FP64"
        results[mode] = r
        print(f"# {mode}: {r}", file=sys.stderr, flush=True)
    if args.copy_probe:
        import torch as _t
        a = _t.empty(args.copy_probe * (1 << 20) // 8, dtype=_t.float64, device="cuda")
        b = _t.empty_like(a)
        a.fill_(1.0)
        for _ in range(5):
            b.copy_(a)
        _t.cuda.synchronize()
        print(f"# copy probe: 5 copies of {a.numel() * 8} bytes", file=sys.stderr, flush=True)
    head = results.get("exhaustive") or results[modes[0]]
    kern_us = head["force_kernel_us"]
    # the dominant kernel: with staged lists, the force kernel that also
    # takes the integrator step (all steps between rebuilds), else the
    # force kernel
    dom_us = head["fused_kernel_us"] or kern_us
    dom_name = head["config"] + (" (force kernel with the fused integrator step)"
                                 if head["fused_kernel_us"] else "")
    line = {
        "metric": "Mpairs/s + us/force step, LJ 1M atoms rho=0.75; learned vs exhaustive vs fixed order",
        "value": head["mpairs_per_s"],
        "unit": "Mpairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "us_per_force_step": kern_us,
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "1M-particle LJ 12-6, FCC 50x50x100 rho=0.75 jitter 0.05, T=1.0, "
                        "rc=2.5, skin=0.3, rebuild every 10, dt=0.002, velocity-Verlet MD steps",
            "particles": n,
            "useful_pairs": pairs,
            "precision": "FP32 pair arithmetic, FP64 accumulation",
            "chosen": head["config"],
            "pruned_inner_list": bool(args.prune),
        },
        "modes": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                  for k, v in results.items()},
    }
    bound, other = rooflines(FLOP_PER_PAIR * pairs, dom_us, head.get("list_stream_bytes"))
    line["roofline"] = dict(bound, **{
        "traffic": measured_traffic(head["config"], head["fused_kernel_us"] is not None),
        "traffic_unit": "HBM bytes per launch (FETCH_SIZE x 2 + WRITE_SIZE x 1, "
                        "factors from a 1 GiB copy)",
        "kernel": dom_name,
        "kernel_us": dom_us})
    if other is not None:
        line["roofline_other"] = other
    if "exhaustive" in results:
        line["tuning_table_us"] = {name: (None if not np.isfinite(v) else round(float(v), 2))
                                   for name, v in zip(space, table)}
    if not args.no_cpu:
        t_step, reps, nth = cpu_baseline(s, args.cpu_seconds)
        import oracle
        t0 = time.perf_counter()
        oracle.forces(s["pos"], s["box"], s["rc"], nthreads=1)
        t_one = time.perf_counter() - t0
        line["cpu_baseline"] = {
            "value": pairs / t_step / 1e6,
            "unit": "Mpairs/s",
            "cores": nth,
            "kind": "oracle",
            "sample": f"{reps} full force evaluations of the same 1M-particle scene "
                      f"(FP64 linked-cell oracle, {t_step:.2f} s each)",
            "threads_used": nth,
            "physical_cores_available": physical_cores(),
            "logical_cpus_available": len(os.sched_getaffinity(0)),
            "host_logical_cpus": os.cpu_count(),
            "one_core": {"value": pairs / t_one / 1e6, "unit": "Mpairs/s", "cores": 1,
                         "sample": f"1 full force evaluation ({t_one:.2f} s)"},
            "cpu_model": cpu_model(),
            "other_scenes": other_oracle_timings(nth),
        }
    sysm.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
