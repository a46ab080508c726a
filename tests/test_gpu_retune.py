"""The dynamic-density workloads with runtime re-tuning, shortened: every
mode runs, tunes at the start and re-checks the scene features between
blocks; on the droplet (Poisson-disk sampled) the tuned modes end on a
configuration far faster than the fixed one-order baseline; the exploding
block's occupancy spread changes between blocks."""
import pytest

pytestmark = pytest.mark.gpu


def test_droplet_retune_blocks_short():
    from paper_2512_03565_amd import retune_demo
    scene = retune_demo.make_scene("droplet", 200_000, 20.0)
    out = {mode: retune_demo.run(mode, steps=300, every=100, samples=4, scene=scene)
           for mode in ("fixed", "exhaustive", "learned", "early_stop")}
    for mode, r in out.items():
        print(f"[retune] {mode}: {r['ms_per_step_incl_tuning']:.3f} ms/step, "
              f"{r['retunes']} tunings, last {r['blocks'][-1]['config']}", flush=True)
        assert len(r["blocks"]) == 3 and r["blocks"][0]["retuned"]
    fixed = out["fixed"]["blocks"][-1]["ms_per_step"]
    for mode in ("exhaustive", "learned", "early_stop"):
        assert out[mode]["blocks"][-1]["ms_per_step"] < 0.7 * fixed, mode


def test_exploding_block_features_move():
    from paper_2512_03565_amd import retune_demo
    scene = retune_demo.make_scene("explode", 128_000)
    r = retune_demo.run("early_stop", steps=600, every=200, samples=2, scene=scene)
    cv = [b["features"]["occupancy_cv"] for b in r["blocks"]]
    print(f"[explode] occupancy cv by block {cv}, retunes {r['retunes']}", flush=True)
    assert len(r["blocks"]) == 3 and r["blocks"][0]["retuned"]
    assert abs(cv[-1] - cv[0]) > 0.01 * cv[0]
