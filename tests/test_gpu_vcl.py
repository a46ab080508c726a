"""GPU parity of the Verlet-cluster-list kernels (cluster size 4 and 8,
cluster-tile orders of both tile shapes and i-per-lane, with and without
Newton-3) against the FP64 oracle, including small and sparse periodic boxes
where a cluster pair is seen through several images."""
import numpy as np
import pytest

from paper_2512_03565_amd import scenes
from tests import _parity as P
from tests.test_gpu_vl import check

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def m():
    from paper_2512_03565_amd import mdlj
    return mdlj


def vcl_configs(m):
    out = []
    for M in (4, 8):
        for n3 in (0, 1):
            out.append((m.NBR_VCL, m.ORD_I_PER_LANE, 0, 0, M, n3))
            # one cluster pair per wavefront (M x 64/M lanes) and 64/(4M)
            # pairs per wavefront (M x 4 lanes each), j or i fastest
            for aj in (64 // M, 4):
                out.append((m.NBR_VCL, m.ORD_CLUSTER_TILE, M, aj, M, n3))
                out.append((m.NBR_VCL, m.ORD_CLUSTER_TILE, M, aj, M, n3, 0, 1))
    return out


def test_vcl_config1(m, orc):
    check(m, orc, scenes.config1(), vcl_configs(m), "cfg1")


def test_vcl_two_species(m, orc):
    check(m, orc, scenes.config4(ncell=12), vcl_configs(m), "2-species")


def test_vcl_config2_100k(m, orc):
    check(m, orc, scenes.config2(), vcl_configs(m), "cfg2")


def test_vcl_sparse_small_box(m, orc):
    box = np.array([17.0, 13.0, 11.0])
    pos = scenes.random_box(200, box, seed=41)
    keep = [0]
    for k in range(1, len(pos)):
        d = pos[keep] - pos[k]
        d -= box * np.rint(d / box)
        if (d * d).sum(1).min() > 0.64:
            keep.append(k)
    s = dict(pos=pos[keep], box=box, rc=2.5, eps=[1.0], sig=[1.0], types=np.zeros(len(keep), np.int32))
    check(m, orc, s, vcl_configs(m), "sparse")


def test_vcl_refresh_and_vv(m, orc):
    import torch
    s = scenes.config1()
    p_ref, v_ref, f_ref, ep, ek = orc.vv(s["pos"], s["vel"], s["box"], s["rc"], s["dt"], 10)
    for cfg in ((m.NBR_VCL, m.ORD_CLUSTER_TILE, 8, 8, 8, 1), (m.NBR_VCL, m.ORD_I_PER_LANE, 0, 0, 4, 0)):
        with m.System(s["pos"], s["box"], s["rc"], skin=0.3, rebuild_every=4, precision=1) as sysm:
            sysm.set_config(cfg)
            vel = [torch.tensor(np.ascontiguousarray(s["vel"][:, k]), device="cuda") for k in range(3)]
            sysm.step_vv(vel, s["dt"], 10)
            f, U, W = sysm.forces()
            pos = sysm.get_positions()
        d = pos - p_ref
        d -= s["box"] * np.rint(d / s["box"])
        assert np.abs(d).max() < 1e-10, cfg
        assert P.force_error(f, f_ref) < 1e-9, cfg
        assert U == pytest.approx(ep[-1], rel=1e-10)
