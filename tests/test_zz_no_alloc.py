"""The allocation-free force call (mdlj_compute_forces_noalloc) against
mdlj_compute_forces: same kernels, so the same forces, energy and virial
bit for bit, on two calls in a row on one GPU (the second on a smaller
context, over the scratch array the first left behind), and its refusals:
a context whose buffers were never sized, and energy partials beyond the
scratch array."""
import numpy as np
import pytest

from paper_2512_03565_amd import scenes
from tests import _parity as P

TOL = {0: 1e-5, 1: 1e-12}

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def m():
    from paper_2512_03565_amd import mdlj
    return mdlj


def same(ref, out, U, W, U2, W2, cfg, prec):
    # Newton-3 kernels add j-forces with atomics, in an order that differs
    # from launch to launch: equal to the parity bar there, bit for bit
    # everywhere else
    if cfg[5]:
        f = np.stack([t.cpu().numpy() for t in out], 1)
        fr = np.stack([t.cpu().numpy() for t in ref], 1)
        assert P.force_error(f, fr) <= TOL[prec], cfg
        assert abs(U2 - U) <= TOL[prec] * abs(U) and abs(W2 - W) <= TOL[prec] * abs(W), cfg
        return
    import torch
    for a, b in zip(ref, out):
        assert torch.equal(a, b), cfg
    assert (U2, W2) == (U, W), cfg


def run_pair(m, s, cfg, prec):
    import torch
    n = len(s["pos"])
    types = s.get("types") if len(s["eps"]) > 1 else None
    with m.System(s["pos"], s["box"], s["rc"], s["eps"], s["sig"], types=types, skin=0.3,
                  precision=prec) as sysm:
        sysm.set_config(cfg)
        ref = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(3)]
        _, U, W = sysm.forces(out=ref)
        # same positions: the structure is current; then moved positions:
        # list upkeep (or re-binning) inside the allocation-free call
        out = [torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
               for _ in range(3)]
        _, U2, W2 = sysm.forces_noalloc(out)
        same(ref, out, U, W, U2, W2, cfg, prec)
        rng = np.random.default_rng(5)
        moved = s["pos"] + rng.uniform(-0.02, 0.02, s["pos"].shape)
        sysm.set_positions(moved)
        _, U3, W3 = sysm.forces_noalloc(out)
        sysm.set_positions(moved)
        _, U4, W4 = sysm.forces(out=ref)
        same(ref, out, U4, W4, U3, W3, cfg, prec)
    return U


@pytest.mark.parametrize("prec,cfg", [(0, (1, 2, 16, 4, 0, 0, 1)), (1, (1, 2, 4, 16, 0, 1)),
                                      (0, (0, 1, 16, 4, 0, 0, 1)), (1, (2, 1, 4, 16, 4, 0))])
def test_noalloc_equals_compute_forces_on_two_calls(m, prec, cfg):
    print(f"[no-alloc] cfg={cfg} prec={prec}: 100k then 1k particles", flush=True)
    run_pair(m, scenes.config2(), cfg, prec)
    run_pair(m, scenes.config1(), cfg, prec)


def test_noalloc_refuses_unsized_context(m):
    import torch
    s = scenes.config1()
    n = len(s["pos"])
    out = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(3)]
    with m.System(s["pos"], s["box"], s["rc"], skin=0.3) as sysm:
        sysm.set_config((1, 2, 16, 4, 0, 0, 1))
        with pytest.raises(m.MdljError) as ei:
            sysm.forces_noalloc(out)
        assert ei.value.status == -4, str(ei.value)
        assert "allocation-free" in str(ei.value)
        # one ordinary call sizes the context; then the allocation-free one works
        ref = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(3)]
        _, U, W = sysm.forces(out=ref)
        _, U2, W2 = sysm.forces_noalloc(out)
        for a, b in zip(ref, out):
            assert torch.equal(a, b)
        assert (U2, W2) == (U, W)


def test_noalloc_refuses_partials_beyond_scratch(m):
    import torch
    # 2.1M particles, Verlet lists with one i per lane: the energy partials
    # (one per wavefront, bounded by n + 64) exceed the 2^22 doubles
    pos, box = scenes.fcc_lattice(64, 64, 128, 0.75, 0.05, seed=7)
    n = len(pos)
    assert 2 * (n + 64) > (1 << 22)
    out = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(3)]
    with m.System(pos, box, 2.5, skin=0.3) as sysm:
        sysm.set_config((1, 0, 0, 0, 0, 0))
        sysm.forces(out=out)
        with pytest.raises(m.MdljError) as ei:
            sysm.forces_noalloc(out)
        assert ei.value.status == -1, str(ei.value)
        assert "scratch" in str(ei.value)
        # forces alone need no partials
        sysm.forces_noalloc(out, energy=False)
