"""Timing sweep that feeds the learned tuner.

For scenes `start .. start+count-1` of ``scenes.tuning_scene`` (seeded), build
the system on the GPU, read the eight scene features from the library and
run the exhaustive tuner, which times every valid configuration.  Writes an
.npz with features [S, 8], amortised step microseconds [S, K] (inf where a
configuration does not apply), the configuration names and scene metadata.

    python -m paper_2512_03565_amd.sweep --start 0 --count 2000 --out sweep.npz

With --configs NAME,NAME,... only those configurations are timed (each one
set and measured like the full search measures it); the other columns are
+inf.  Tables of the same scenes are merged column by column by
``train_tuner.load``.
"""
import argparse
import sys
import time

import numpy as np


def run(start, count, samples, out, n_max, only=None):
    import torch  # noqa: F401  (one HIP runtime: torch's)
    from paper_2512_03565_amd import mdlj, scenes
    feats, tables, meta = [], [], []
    names = None
    t0 = time.time()
    for k in range(start, start + count):
        s = scenes.tuning_scene(k, n_max=n_max)
        types = s["types"] if len(s["eps"]) > 1 else None
        try:
            with mdlj.System(s["pos"], s["box"], s["rc"], s["eps"], s["sig"], types=types,
                             skin=s["skin"], rebuild_every=s["rebuild_every"]) as sysm:
                if names is None:
                    names = [mdlj.config_name(c) for c in sysm.configs()]
                f = sysm.features()
                if only:
                    cfgs = sysm.configs()
                    tab = np.full(len(cfgs), np.inf)
                    for name in only:
                        j = names.index(name)
                        sysm.set_config(cfgs[j])
                        try:
                            tab[j] = sysm.tune(mdlj.TUNE_FIXED, samples)[1]
                        except mdlj.MdljError:
                            pass  # not valid for this scene
                else:
                    sysm.tune(mdlj.TUNE_EXHAUSTIVE, samples)
                    tab = sysm.tune_results()
        except mdlj.MdljError as e:
            print(f"scene {k}: skipped ({e})", flush=True)
            continue
        feats.append(f)
        tables.append(tab)
        meta.append((k, len(s["pos"]), s["rho"], s["rc"], len(s["eps"]), int(s["droplet"])))
        if (k - start) % 10 == 0 or k == start + count - 1:
            best = names[int(np.argmin(tab))]
            print(f"[sweep] scene {k} n={len(s['pos'])} best={best} {np.min(tab):.1f}us "
                  f"elapsed {time.time() - t0:.0f}s", flush=True)
    np.savez(out, features=np.array(feats, np.float32), table_us=np.array(tables),
             names=np.array(names), meta=np.array(meta, np.float64))
    print(f"wrote {out}: {len(feats)} scenes", flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--start", type=int, default=0)
    ap.add_argument("--count", type=int, default=2000)
    ap.add_argument("--samples", type=int, default=4)
    ap.add_argument("--n-max", type=float, default=4e6)
    ap.add_argument("--out", default="sweep.npz")
    ap.add_argument("--configs", default=None, help="comma-separated configuration names")
    a = ap.parse_args(argv)
    run(a.start, a.count, a.samples, a.out, a.n_max,
        a.configs.split(",") if a.configs else None)
    return 0


if __name__ == "__main__":
    sys.exit(main())
