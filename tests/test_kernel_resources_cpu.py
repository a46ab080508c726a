"""Register budget of the staged Verlet-list force kernels (no GPU): the
fused-step variant is held to 64 VGPRs so that eight wavefronts share a
SIMD, and no force kernel of vl.hip may spill to scratch (a spill in the
fused kernel once cost it 40% of its speed).  Compiles vl.hip for gfx950
with the library's own flags and reads the code-object metadata."""
import os
import re
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "paper_2512_03565_amd"))


@pytest.fixture(scope="module")
def kernels(tmp_path_factory):
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    import build
    out = str(tmp_path_factory.mktemp("asm") / "vl.s")
    cmd = ["hipcc", "-x", "hip", *build.COMMON, "--cuda-device-only", "-S",
           os.path.join(build.CSRC, "vl.hip"), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    text = open(out).read()
    res = {}
    for blk in text.split("  - .agpr_count:")[1:]:
        name = re.search(r"\.name:\s+(\S+)", blk).group(1)
        res[name] = (int(re.search(r"\.vgpr_count:\s+(\d+)", blk).group(1)),
                     int(re.search(r"\.vgpr_spill_count:\s+(\d+)", blk).group(1)),
                     int(re.search(r"\.sgpr_spill_count:\s+(\d+)", blk).group(1)))
    return res


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
