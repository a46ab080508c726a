"""The kernels' lane -> (i, j) maps against the register fills of the
paper's four interaction orders (section 4.1.1, Fig. "vec_patterns"; the
8-way fills are in tests/golden/register_fills_8.json), and their 64-lane
forms per configuration.  No GPU: the library exports the maps its kernels
use as host functions."""
import json
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "register_fills_8.json")


@pytest.fixture(scope="module")
def m():
    from paper_2512_03565_amd import mdlj
    return mdlj


@pytest.mark.parametrize("name,layout,ai", [("1/8", 0, 1), ("2/4", 0, 2), ("8/1", 1, 8),
                                            ("4/2", 1, 4)])
def test_eight_way_fills_match_the_figure(m, name, layout, ai):
    g = json.load(open(GOLDEN))[name]
    i, j = m.lane_map(layout, ai, 8)
    assert list(i) == g["i"] and list(j) == g["j"]


def test_the_two_layouts_are_transposes(m):
    for ai in (1, 2, 4, 8, 16, 32, 64):
        i0, j0 = m.lane_map(0, ai, 64)
        i1, j1 = m.lane_map(1, 64 // ai, 64)
        # i fastest with 64/ai i's covers the transposed grid of j fastest
        assert sorted(zip(i0, j0)) == sorted(zip(j1, i1))


def _grid_ok(i, j, ai):
    aj = 64 // ai
    pairs = set(zip(i.tolist(), j.tolist()))
    return len(pairs) == 64 and pairs == {(a, b) for a in range(ai) for b in range(aj)}


CASES = [
    # (configuration, layout, i's per step) and which fill it widens
    ((0, 0, 1, 1, 0, 0, 0), 1, 64),        # LC i-per-lane: VectorLength/1
    ((0, 2, 1, 64, 0, 0, 1), 0, 1),        # LC wave-per-i 1x64: 1/VectorLength
    ((0, 2, 2, 32, 0, 0, 0), 0, 2),        # LC wave-per-i 2x32: 2/(VL/2)
    ((0, 1, 16, 4, 0, 0, 1), 0, 16),       # LC cluster tile 16x4
    ((0, 1, 4, 16, 0, 1, 1, 0), 0, 4),     # LC Newton 3 cluster tile 4x16
    ((0, 0, 1, 1, 0, 1, 1, 1), 1, 64),     # LC Newton 3, roles swapped
    ((1, 0, 0, 0, 0, 0), 1, 64),           # VL i-per-lane
    ((1, 2, 16, 4, 0, 0, 1), 0, 16),       # staged VL 16 i's x 4 lanes
    ((2, 1, 4, 16, 4, 0), 0, 4),           # VCL4 tile, j fastest: 2/(VL/2) widened
    ((2, 1, 4, 16, 4, 0, 0, 1), 1, 4),     # VCL4 tile, i fastest: (VL/2)/2 widened
    ((2, 1, 8, 8, 8, 1, 0, 1), 1, 8),      # VCL8 tile, i fastest
    ((2, 0, 0, 0, 8, 0), 1, 64),           # VCL8 i-per-lane
]


@pytest.mark.parametrize("cfg,layout,ai", CASES)
def test_configuration_lane_maps(m, cfg, layout, ai):
    lay, i, j = m.config_lane_map(cfg)
    assert lay == layout
    assert _grid_ok(i, j, ai)
    ei, ej = m.lane_map(layout, ai, 64)
    assert np.array_equal(i, ei) and np.array_equal(j, ej)
    # the 8-way fill of the same shape is the first 8 lanes' pattern for
    # ai = 1 (1/VL) and ai = 64 (VL/1)
    if ai == 1:
        assert list(i[:8]) == [0] * 8 and list(j[:8]) == list(range(8))
    if ai == 64:
        assert list(i[:8]) == list(range(8)) and list(j[:8]) == [0] * 8


# VCL tiles with several cluster pairs per wavefront: (configuration, layout,
# cluster size, j-lanes per pair)
GROUPED = [
    ((2, 1, 4, 4, 4, 0), 0, 4, 4),         # VCL4 4x4 x 4 pairs, j fastest
    ((2, 1, 4, 4, 4, 1, 0, 1), 1, 4, 4),   # the same, i fastest, Newton 3
    ((2, 1, 8, 4, 8, 0), 0, 8, 4),         # VCL8 8x4 x 2 pairs, j fastest
    ((2, 1, 8, 4, 8, 0, 0, 1), 1, 8, 4),   # the same, i fastest
]


@pytest.mark.parametrize("cfg,layout,M,aj", GROUPED)
def test_grouped_cluster_tile_lane_maps(m, cfg, layout, M, aj):
    lay, i, j = m.config_lane_map(cfg)
    assert lay == layout
    w = M * aj
    q = np.arange(64) // w
    # each group of w lanes is one cluster pair: its own M i's and aj j-lanes
    assert np.array_equal(i // M, q) and np.array_equal(j // aj, q)
    # every (i, j) of each group's M x aj block exactly once
    blocks = {(g * M + a, g * aj + b) for g in range(64 // w) for a in range(M) for b in range(aj)}
    assert set(zip(i.tolist(), j.tolist())) == blocks and len(blocks) == 64
    # inside a group, the one-pair map at width w
    ei, ej = m.lane_map(layout, M, w)
    for g in range(64 // w):
        sl = slice(g * w, (g + 1) * w)
        assert np.array_equal(i[sl] - g * M, ei) and np.array_equal(j[sl] - g * aj, ej)
    # 4 j-lanes per pair, j fastest: the first 8 lanes are the 2/(VL/2) fill
    # of the figure
    if layout == 0:
        g8 = json.load(open(GOLDEN))["2/4"]
        assert list(i[:8]) == g8["i"] and list(j[:8]) == g8["j"]


def test_lane_map_rejects_bad_shapes(m):
    with pytest.raises(m.MdljError):
        m.lane_map(0, 3, 8)
    with pytest.raises(m.MdljError):
        m.lane_map(2, 1, 8)


def test_cluster_tile_names(m):
    # one cluster pair per wavefront: M x 64/M; several: M x 4 x (pairs)
    assert m.config_name((2, 1, 4, 16, 4, 0)) == "VCL4/cluster-tile/4x16"
    assert m.config_name((2, 1, 8, 8, 8, 1, 0, 1)) == "VCL8/cluster-tile/8x8/n3/swap"
    assert m.config_name((2, 1, 4, 4, 4, 0)) == "VCL4/cluster-tile/4x4x4"
    assert m.config_name((2, 1, 8, 4, 8, 1, 0, 1)) == "VCL8/cluster-tile/8x4x2/n3/swap"
    # linked-cell tiles keep their two-number names
    assert m.config_name((0, 1, 16, 4, 0, 0, 1)) == "LC/cluster-tile/16x4/lds"
