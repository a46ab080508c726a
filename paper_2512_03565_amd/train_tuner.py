"""Train the learned tuner on sweep timings and score it on held-out scenes.

Reads one or more sweep .npz files (``sweep.py``), labels every scene with
its fastest configuration, z-scores the features on the training scenes,
trains the network on the GPU with the library's own kernels and evaluates
the held-out scenes:

  regret(scene) = t(chosen) / t(fastest) with both times from the sweep,
  chosen = the network's argmax when its confidence >= threshold, else full
  search (which picks the fastest, regret 1, but pays for timing every
  configuration).

Writes the network file and a JSON summary.

    python -m paper_2512_03565_amd.train_tuner sweep_a.npz sweep_b.npz \
        --out paper_2512_03565_amd/data/tuner_mlp.bin
"""
import argparse
import json
import sys

import numpy as np


def load(paths):
    """Features, tables, metadata and configuration names of the sweeps,
    one row per scene (by scene index).  Columns are matched by
    configuration name: the longest name list is the space; a sweep of the
    same scenes that timed other (or the same) configurations fills their
    columns, a later file's finite value replacing an earlier one (so a
    re-timing of some configurations after a kernel change goes last)."""
    data = [np.load(p, allow_pickle=False) for p in paths]
    names = max((list(d["names"]) for d in data), key=len)
    rows = {}
    for d in data:
        cols = [names.index(nm) for nm in list(d["names"])]
        for f, t, mt in zip(d["features"], d["table_us"], d["meta"]):
            sid = int(mt[0])
            if sid not in rows:
                rows[sid] = [f, np.full(len(names), np.inf), mt]
            row = rows[sid][1]
            for c, v in zip(cols, t):
                if np.isfinite(v):
                    row[c] = v
    sids = sorted(rows)
    F = np.array([rows[s][0] for s in sids], np.float32)
    T = np.array([rows[s][1] for s in sids])
    M = np.array([rows[s][2] for s in sids], np.float64)
    return F, T, M, names


def best_fixed(table, names):
    """The single configuration with the smallest geometric-mean
    t(config) / t(fastest) over the rows of table (configurations that cannot
    run on some scene are left out): what one fixed choice gets."""
    best = np.min(table, axis=1)
    ok = np.isfinite(table).all(0)
    g = np.full(table.shape[1], np.inf)
    g[ok] = np.exp(np.log(table[:, ok] / best[:, None]).mean(0))
    k = int(np.argmin(g))
    return k, names[k], float(g[k])


def evaluate(probs, table, threshold):
    best = np.min(table, axis=1)
    pick = probs.argmax(1)
    conf = probs.max(1)
    t_pick = table[np.arange(len(table)), pick]
    fallback = (conf < threshold) | ~np.isfinite(t_pick)
    ratio = np.where(fallback, 1.0, t_pick / best)
    return {
        "geomean_ratio": float(np.exp(np.log(ratio).mean())),
        "mean_ratio": float(ratio.mean()),
        "max_ratio": float(ratio.max()),
        "fallback_rate": float(fallback.mean()),
        "top1_accuracy": float((pick == table.argmin(1)).mean()),
        "within_5pct": float((ratio <= 1.05).mean()),
    }


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("sweeps", nargs="+")
    ap.add_argument("--train", type=int, default=1600, help="first N scenes train, rest test")
    ap.add_argument("--epochs", type=int, default=200)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=20251203)
    ap.add_argument("--threshold", type=float, default=0.6)
    ap.add_argument("--out", default="tuner_mlp.bin")
    ap.add_argument("--summary", default=None)
    ap.add_argument("--save-sweep", default=None,
                    help="also write the merged sweep (one row per scene) to this .npz")
    a = ap.parse_args(argv)

    import torch  # noqa: F401  (one HIP runtime: torch's)
    from paper_2512_03565_amd import mdlj, scenes

    F, T, meta, names = load(a.sweeps)
    if a.save_sweep:
        np.savez_compressed(a.save_sweep, features=F, table_us=T, names=np.array(names),
                            meta=meta)
    ok = np.isfinite(T).any(1)
    F, T, meta = F[ok], T[ok], meta[ok]
    y = T.argmin(1).astype(np.int32)
    ntr = min(a.train, len(F) - 1)
    Ftr, ytr = F[:ntr], y[:ntr]
    mean = Ftr.mean(0)
    std = Ftr.std(0)
    std[std < 1e-6] = 1.0
    s = scenes.config1()
    with mdlj.System(s["pos"], s["box"], s["rc"]) as sysm:
        if [mdlj.config_name(c) for c in sysm.configs()] != names:
            raise ValueError("sweep configurations differ from the library's configuration space")
        sysm.mlp_init(T.shape[1], seed=a.seed)
        sysm.mlp_set_norm(mean, std)
        loss = sysm.mlp_train(Ftr, ytr, a.epochs, a.batch, a.lr, a.seed + 1)
        sysm.mlp_set_threshold(a.threshold)
        sysm.mlp_save(a.out)
        p_tr = sysm.mlp_predict(Ftr)
        p_te = sysm.mlp_predict(F[ntr:])
    fixed = names.index("LC/i-per-lane/k1")
    kb, name_b, _ = best_fixed(T[:ntr], names)
    res = {
        "scenes": int(len(F)), "train": int(ntr), "test": int(len(F) - ntr),
        "configs": names, "final_loss": loss, "threshold": a.threshold,
        "train_eval": evaluate(p_tr, T[:ntr], a.threshold),
        "test_eval": evaluate(p_te, T[ntr:], a.threshold),
        "test_fixed_geomean_ratio": float(np.exp(np.log(T[ntr:, fixed] / T[ntr:].min(1)).mean())),
        "best_single_config": name_b,
        "test_best_single_geomean_ratio": float(np.exp(np.log(T[ntr:, kb] / T[ntr:].min(1)).mean())),
        "label_histogram": {names[k]: int(c) for k, c in zip(*np.unique(y, return_counts=True))},
    }
    print(json.dumps(res["test_eval"]), flush=True)
    if a.summary:
        with open(a.summary, "w") as f:
            json.dump(res, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
