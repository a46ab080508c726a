"""Score a trained tuner network on held-out scenes with fresh GPU timings.

For every held-out scene of the sweep (scene index >= --first), on the GPU:

  * learned tuning: features -> network -> the predicted configuration is
    timed (or, below the confidence threshold, the full search runs); the
    wall time of the tuning call is recorded;
  * both the learned choice and the sweep's fastest configuration are timed
    again with --samples samples each (amortised step time, the tuner's own
    objective), and regret = t(learned) / t(fastest) - 1;
  * the fixed one-order baseline (linked cells, i-per-lane) and the best
    single configuration of the training scenes (smallest geometric-mean
    step-time ratio to the fastest over the sweep's training rows) are
    timed the same way;
  * the early-stopping search runs (visiting configurations in the
    network's order) and its choice is timed the same way;
  * on every --full-every-th scene the full search is run as well, for the
    cost of tuning without the network.

Writes a JSON summary.

    python -m paper_2512_03565_amd.eval_tuner sweep_0.npz sweep_1000.npz \
        --weights paper_2512_03565_amd/data/tuner_mlp.bin --out eval.json

Offline (no GPU), after some configurations were timed again on the
held-out scenes (``sweep.py --configs``): the sweep-table regret of the
decisions an evaluation recorded, against the sweep's timings and against
the same timings with the re-timed columns replaced.

    python -m paper_2512_03565_amd.eval_tuner paper_2512_03565_amd/data/tuner_sweep.npz \
        --retimed paper_2512_03565_amd/data/tuner_sweep_vcl_heldout.npz \
        --decisions paper_2512_03565_amd/data/tuner_eval.json
"""
import argparse
import json
import sys
import time

import numpy as np


def retimed_regret(names, table, sids, retimed, decisions):
    """Sweep-table regret t(decision) / t(fastest) of recorded decisions,
    before and after replacing the columns `retimed` holds (finite values
    only) for the scenes it holds.  names, table [S, K] and sids describe
    the sweep; retimed is (names, table, sids) of the re-timing; decisions
    are the evaluation's scene records (a fallback ran the full search,
    which finds the fastest: regret 0).  Returns per-scene ratios (before,
    after) and the number of scenes whose fastest configuration changed."""
    row = {int(s): k for k, s in enumerate(sids)}
    rnames, rtable, rsids = retimed
    cols = [names.index(n) for n in rnames]
    rrow = {int(s): k for k, s in enumerate(rsids)}
    before, after, changed = [], [], 0
    for d in decisions:
        sid = int(d["scene"])
        if sid not in row or sid not in rrow:
            continue
        t0 = np.asarray(table[row[sid]], float)
        t1 = t0.copy()
        for c, v in zip(cols, rtable[rrow[sid]]):
            if np.isfinite(v):
                t1[c] = v
        changed += int(np.argmin(t1) != np.argmin(t0))
        if d["fallback"]:
            before.append(1.0)
            after.append(1.0)
        else:
            c = names.index(d["chosen"])
            before.append(t0[c] / t0.min())
            after.append(t1[c] / t1.min())
    return np.array(before), np.array(after), changed


def offline(a):
    from paper_2512_03565_amd.train_tuner import load
    F, T, meta, names = load(a.sweeps)
    r = np.load(a.retimed, allow_pickle=False)
    with open(a.decisions) as f:
        dec = json.load(f)["scenes"]
    b, c, changed = retimed_regret(names, T, meta[:, 0], (list(r["names"]), r["table_us"],
                                                            r["meta"][:, 0]), dec)
    g = lambda x: float(np.exp(np.log(x).mean()) - 1)
    print(json.dumps({"scenes": int(len(b)), "fastest_changed": changed,
                      "regret_geomean_before": g(b), "regret_geomean_after": g(c),
                      "within_5pct_before": float((b <= 1.05).mean()),
                      "within_5pct_after": float((c <= 1.05).mean()),
                      "regret_max_before": float(b.max() - 1),
                      "regret_max_after": float(c.max() - 1)}), flush=True)
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("sweeps", nargs="+")
    ap.add_argument("--weights", default=None)
    ap.add_argument("--retimed", default=None, help="offline: re-timed columns (.npz)")
    ap.add_argument("--decisions", default=None, help="offline: an evaluation's JSON")
    ap.add_argument("--first", type=int, default=1600, help="first held-out scene index")
    ap.add_argument("--count", type=int, default=400)
    ap.add_argument("--samples", type=int, default=10)
    ap.add_argument("--tune-samples", type=int, default=4)
    ap.add_argument("--full-every", type=int, default=4)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    if a.retimed:
        if not a.decisions:
            ap.error("--retimed needs --decisions")
        return offline(a)
    if not a.weights:
        ap.error("--weights is required")

    import torch  # noqa: F401  (one HIP runtime: torch's)
    from paper_2512_03565_amd import mdlj, scenes
    from paper_2512_03565_amd.train_tuner import load

    from paper_2512_03565_amd.train_tuner import best_fixed
    F, T, meta, names = load(a.sweeps)
    train_rows = [k for k in range(len(meta)) if meta[k, 0] < a.first]
    kb, name_b, _ = best_fixed(T[train_rows], names)
    idx = [k for k in range(len(meta)) if meta[k, 0] >= a.first][: a.count]
    rows = []
    t0 = time.time()
    for q, k in enumerate(idx):
        sid = int(meta[k, 0])
        s = scenes.tuning_scene(sid)
        types = s["types"] if len(s["eps"]) > 1 else None
        with mdlj.System(s["pos"], s["box"], s["rc"], s["eps"], s["sig"], types=types,
                         skin=s["skin"], rebuild_every=s["rebuild_every"]) as sysm:
            space = [mdlj.config_name(c) for c in sysm.configs()]
            # the sweep covers the library's space, or the part of it that
            # existed when it was taken (configurations are only appended)
            if space[:len(names)] != names:
                raise ValueError("sweep and library configuration spaces differ")
            cfgs = sysm.configs()
            sysm.mlp_load(a.weights)
            _, fb0 = sysm.mlp_stats()
            c0 = time.perf_counter()
            chosen, _ = sysm.tune(mdlj.TUNE_LEARNED, a.tune_samples)
            t_learn = time.perf_counter() - c0
            conf, fb1 = sysm.mlp_stats()
            ci = space.index(mdlj.config_name(chosen))
            best = int(np.argmin(T[k]))

            def timed(j):
                sysm.set_config(cfgs[j])
                return sysm.tune(mdlj.TUNE_FIXED, a.samples)[1]

            us_l = timed(ci)
            us_b = us_l if best == ci else timed(best)
            us_f = timed(space.index("LC/i-per-lane/k1"))
            us_s = timed(kb)
            c0 = time.perf_counter()
            early, _ = sysm.tune(mdlj.TUNE_EARLY_STOP, a.tune_samples)
            t_early = time.perf_counter() - c0
            taken_early = int(sysm.tune_taken().sum())
            ei = space.index(mdlj.config_name(early))
            us_e = us_l if ei == ci else (us_b if ei == best else timed(ei))
            t_full = None
            if q % a.full_every == 0:
                c0 = time.perf_counter()
                sysm.tune(mdlj.TUNE_EXHAUSTIVE, a.tune_samples)
                t_full = time.perf_counter() - c0
        rows.append(dict(scene=sid, n=int(meta[k, 1]), chosen=space[ci], best=space[best],
                         confidence=conf, fallback=bool(fb1 > fb0), us_learned=us_l,
                         us_best=us_b, us_fixed=us_f, us_best_single=us_s,
                         early=space[ei], us_early=us_e, tune_s_early=t_early,
                         samples_early=taken_early, tune_s_learned=t_learn,
                         tune_s_full=t_full))
        if q % 20 == 0:
            print(f"[eval] {q}/{len(idx)} scene {sid} {space[ci]} vs {space[best]} "
                  f"ratio {us_l / us_b:.3f} elapsed {time.time() - t0:.0f}s", flush=True)
    r = np.array([x["us_learned"] / x["us_best"] for x in rows])
    fx = np.array([x["us_fixed"] / x["us_best"] for x in rows])
    bs = np.array([x["us_best_single"] / x["us_best"] for x in rows])
    re = np.array([x["us_early"] / x["us_best"] for x in rows])
    tl = np.array([x["tune_s_learned"] for x in rows])
    full = [x for x in rows if x["tune_s_full"] is not None]
    summary = {
        "scenes": len(rows),
        "samples": a.samples,
        "regret_geomean": float(np.exp(np.log(r).mean()) - 1),
        "regret_mean": float(r.mean() - 1),
        "regret_p90": float(np.percentile(r, 90) - 1),
        "regret_max": float(r.max() - 1),
        "within_5pct": float((r <= 1.05).mean()),
        "fallback_rate": float(np.mean([x["fallback"] for x in rows])),
        "same_as_best": float(np.mean([x["chosen"] == x["best"] for x in rows])),
        "fixed_over_best_geomean": float(np.exp(np.log(fx).mean())),
        "best_single_config": name_b,
        "best_single_over_best_geomean": float(np.exp(np.log(bs).mean())),
        "learned_gain_over_best_single_geomean": float(np.exp(np.log(bs / r).mean())),
        "early_stop_regret_geomean": float(np.exp(np.log(re).mean()) - 1),
        "early_stop_within_5pct": float((re <= 1.05).mean()),
        "tune_s_early_mean": float(np.mean([x["tune_s_early"] for x in rows])),
        "samples_early_mean": float(np.mean([x["samples_early"] for x in rows])),
        "tune_s_learned_mean": float(tl.mean()),
        "tune_s_full_mean": float(np.mean([x["tune_s_full"] for x in full])) if full else None,
        "tune_s_learned_on_full_scenes": float(np.mean([x["tune_s_learned"] for x in full]))
        if full else None,
    }
    print(json.dumps(summary), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump({"summary": summary, "scenes": rows}, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
