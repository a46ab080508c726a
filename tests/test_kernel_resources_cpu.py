"""Register budget of the force kernels (no GPU): the staged Verlet-list
kernel's fused-step variant and the single-species forces-only cluster
tiles are held to 64 VGPRs so that eight wavefronts share a SIMD, and no
force kernel of vl.hip or vcl.hip may spill to scratch (a spill in the
fused kernel once cost it 40% of its speed).  Compiles the sources for
gfx950 with the library's own flags and reads the code-object metadata."""
import os
import re
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "paper_2512_03565_amd"))


def _resources(tmp_path_factory, src):
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    import build
    out = str(tmp_path_factory.mktemp("asm") / (src + ".s"))
    cmd = ["hipcc", "-x", "hip", *build.COMMON, "--cuda-device-only", "-S",
           os.path.join(build.CSRC, src), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    text = open(out).read()
    res = {}
    for blk in text.split("  - .agpr_count:")[1:]:
        name = re.search(r"\.name:\s+(\S+)", blk).group(1)
        res[name] = (int(re.search(r"\.vgpr_count:\s+(\d+)", blk).group(1)),
                     int(re.search(r"\.vgpr_spill_count:\s+(\d+)", blk).group(1)),
                     int(re.search(r"\.sgpr_spill_count:\s+(\d+)", blk).group(1)))
    return res


@pytest.fixture(scope="module")
def kernels(tmp_path_factory):
    return _resources(tmp_path_factory, "vl.hip")


@pytest.fixture(scope="module")
def cluster_kernels(tmp_path_factory):
    return _resources(tmp_path_factory, "vcl.hip")


def test_fused_kernels_fit_64_vgprs_without_spills(kernels):
    w8 = {k: v for k, v in kernels.items() if "k_vl_lds_w8" in k}
    assert len(w8) >= 4
    for name, (vgpr, vspill, sspill) in w8.items():
        assert vgpr <= 64 and vspill == 0 and sspill == 0, (name, vgpr, vspill, sspill)


def test_no_force_kernel_spills(kernels):
    forces = {k: v for k, v in kernels.items() if "k_vl_" in k}
    assert forces
    for name, (vgpr, vspill, sspill) in forces.items():
        assert vspill == 0 and sspill == 0, (name, vgpr, vspill, sspill)


def test_cluster_kernels_do_not_spill(cluster_kernels):
    forces = {k: v for k, v in cluster_kernels.items() if "k_vcl_" in k}
    assert forces
    for name, (vgpr, vspill, sspill) in forces.items():
        assert vspill == 0 and sspill == 0, (name, vgpr, vspill, sspill)


def test_cluster_tiles_keep_eight_wavefronts(cluster_kernels):
    # the single-species forces-only cluster tiles (the form the MD steps
    # run) within 64 registers, so that eight wavefronts share a SIMD: a
    # per-step member index kept live through the pair loop once took them
    # to 84-90 and cost 12-24% of their speed
    tiles = {k: v for k, v in cluster_kernels.items()
             if "k_vcl_tile" in k and ("IfLb0ELb0ELb0E" in k or "IdLb0ELb0ELb0E" in k)}
    assert len(tiles) >= 8
    for name, (vgpr, _, _) in tiles.items():
        assert vgpr <= 64, (name, vgpr)

