"""The droplet workload with runtime re-tuning, shortened: every mode runs,
tunes at the start, re-checks the scene features between blocks and the
learned and full-search modes end on a configuration far faster than the
fixed one-order baseline."""
import pytest

pytestmark = pytest.mark.gpu


def test_droplet_retune_blocks_short():
    from paper_2512_03565_amd import retune_demo
    out = {mode: retune_demo.run(mode, steps=300, every=100, samples=4, n_total=200_000,
                                     r_drop=20.0)
           for mode in ("fixed", "exhaustive", "learned")}
    for mode, r in out.items():
        print(f"[retune] {mode}: {r['ms_per_step_incl_tuning']:.3f} ms/step, "
              f"{r['retunes']} tunings, last {r['blocks'][-1]['config']}", flush=True)
        assert len(r["blocks"]) == 3 and r["blocks"][0]["retuned"]
    fixed = out["fixed"]["blocks"][-1]["ms_per_step"]
    for mode in ("exhaustive", "learned"):
        assert out[mode]["blocks"][-1]["ms_per_step"] < 0.7 * fixed, mode
