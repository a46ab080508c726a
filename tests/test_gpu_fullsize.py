"""Parity at full size, in the launch configurations the benchmark times.

1M-particle headline scene (50x50x100 FCC, rho 0.75, rc 2.5, skin 0.3): the
oracle's linked-cell sum is fast enough to compare every particle, for the
configuration the benchmark runs and the other leading ones, FP32 pair path
and all-FP64 path.  4M-particle two-species scene (rho 0.7, rc 3.0,
Verlet cluster lists with clusters of 4 and 8): forces compared on a seeded
50,000-particle sample with the oracle's per-particle sum, energy and virial
with its full sum.
"""
import numpy as np
import pytest

from paper_2512_03565_amd import scenes
from tests import _parity as P

pytestmark = pytest.mark.gpu

TOL = {0: 1e-5, 1: 1e-12}


@pytest.fixture(scope="module")
def m():
    from paper_2512_03565_amd import mdlj
    return mdlj


def by_name(sysm, m, name):
    names = [m.config_name(c) for c in sysm.configs()]
    return sysm.configs()[names.index(name)]


def test_headline_1m_every_particle(m, orc):
    s = scenes.headline()
    pos, box, rc = s["pos"], s["box"], s["rc"]
    ref = orc.forces(pos, box, rc)
    runs = {0: ["VL/wave-per-i/16x4/lds", "VL/wave-per-i/8x8", "VL/wave-per-i/16x4",
                "LC/cluster-tile/16x4/lds", "VCL4/cluster-tile/4x16", "VL/wave-per-i/16x4/n3",
                "LC/cluster-tile/4x16/n3/lds", "LC/i-per-lane/n3/lds/swap"],
            1: ["VL/wave-per-i/16x4/lds", "LC/i-per-lane/k1", "LC/wave-per-i/1x64/n3/lds",
                "LC/cluster-tile/16x4/n3/lds"]}
    with m.System(pos, box, rc, skin=s["skin"], rebuild_every=s["rebuild_every"]) as sysm:
        for prec, names in runs.items():
            band = P.fx_band(box, rc, s["skin"]) if prec == 0 else P.F64_BAND
            slack, su, sw, namb = P.boundary_slack(orc, pos, box, rc, [1.0], [1.0], None, True,
                                                   band)
            sysm.set_precision(prec)
            for name in names:
                print(f"[fullsize] 1M prec={prec} {name} (ambiguous pairs {namb})", flush=True)
                sysm.set_config(by_name(sysm, m, name))
                f, U, W = sysm.forces()
                e = P.force_error(f, ref["f"], slack)
                assert e <= TOL[prec], (name, prec, e)
                assert P.total_error(U, ref["U"], su) <= TOL[prec], (name, prec, U, ref["U"])
                assert P.total_error(W, ref["W"], sw) <= TOL[prec], (name, prec, W, ref["W"])


def test_config4_4m_two_species_cluster_lists_sampled(m, orc):
    s = scenes.config4()
    pos, box, rc, types = s["pos"], s["box"], s["rc"], s["types"]
    assert len(pos) == 4_000_000
    idx = np.sort(np.random.default_rng(20251205).choice(len(pos), 50_000, replace=False))
    sub = orc.forces_subset(pos, box, rc, idx, s["eps"], s["sig"], types)
    full = orc.forces(pos, box, rc, s["eps"], s["sig"], types)
    assert np.allclose(full["f"][idx], sub["f"], rtol=0, atol=1e-12 * P.frms(full["f"]))
    names = ["VCL4/cluster-tile/4x16", "VCL8/cluster-tile/8x8", "VCL4/i-per-lane",
             "VCL8/i-per-lane/n3", "VCL4/cluster-tile/4x4x4", "VCL8/cluster-tile/8x4x2/n3"]
    with m.System(pos, box, rc, s["eps"], s["sig"], types=types, skin=s["skin"],
                  rebuild_every=s["rebuild_every"]) as sysm:
        for prec in (0, 1):
            band = P.fx_band(box, rc, s["skin"]) if prec == 0 else P.F64_BAND
            slack = P.boundary_slack_subset(orc, pos, box, rc, s["eps"], s["sig"], types, True,
                                            band, idx)
            sysm.set_precision(prec)
            for name in names:
                print(f"[fullsize] 4M prec={prec} {name}", flush=True)
                sysm.set_config(by_name(sysm, m, name))
                f, U, W = sysm.forces()
                e = P.force_error(f[idx], sub["f"], slack, scale=P.frms(full["f"]))
                assert e <= TOL[prec], (name, prec, e)
                # totals: u(rc) = 0 with the shift, so ambiguous pairs do not move U,
                # and their virial is far below these bars
                assert P.total_error(U, full["U"]) <= TOL[prec], (name, prec, U, full["U"])
                assert P.total_error(W, full["W"]) <= TOL[prec], (name, prec, W, full["W"])
