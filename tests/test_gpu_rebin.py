"""Binning when the number of halo images grows between rebuilds: the
records' scatter and fill are queued before the host learns the new total,
into the buffers of the last binning, and must be run again into larger
ones when the total no longer fits.  Forces after the change are compared
with the FP64 oracle (section 2.1, Eq. 1)."""
import numpy as np
import pytest

from tests import _parity as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def m():
    from paper_2512_03565_amd import mdlj
    return mdlj


def _scenes(seed=11):
    rng = np.random.default_rng(seed)
    box = np.full(3, 20.0)
    k = np.arange(9)
    grid = np.stack(np.meshgrid(k, k, k, indexing="ij"), -1).reshape(-1, 3).astype(float)
    # first: every particle in the middle of the box (spacing 1.1), away
    # from the cells next to the faces, so there are no halo images; then:
    # the same number over the whole box (spacing 20/9), with images of
    # about half of them
    inner = 5.6 + 1.1 * grid + rng.uniform(-0.05, 0.05, grid.shape)
    whole = (20.0 / 9.0) * (grid + 0.5) + rng.uniform(-0.1, 0.1, grid.shape)
    return inner, whole, box


@pytest.mark.parametrize("cfg", [(0, 0, 1, 1, 0, 0), (1, 2, 16, 4, 0, 0, 1), (1, 0, 0, 0, 0, 0)])
def test_more_images_after_a_rebuild(m, orc, cfg):
    inner, whole, box = _scenes()
    rc = 2.5
    print(f"[rebin] cfg={cfg}", flush=True)
    with m.System(inner, box, rc, skin=0.3, precision=1) as sysm:
        sysm.set_config(cfg)
        f0, _, _ = sysm.forces()
        ref0 = orc.forces(inner, box, rc)
        assert P.force_error(f0, ref0["f"]) < 1e-12
        for pos in (whole, inner, whole):
            sysm.set_positions(pos)
            f, U, W = sysm.forces()
            ref = orc.forces(pos, box, rc)
            slack, su, sw, _ = P.boundary_slack(orc, pos, box, rc, [1.0], [1.0], None, True,
                                                P.F64_BAND)
            assert P.force_error(f, ref["f"], slack) < 1e-12, cfg
            assert P.total_error(U, ref["U"], su) < 1e-12
