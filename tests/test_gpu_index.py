"""Index work of the neighbour structures against the oracle, bit for bit
(section 2.1.1): the cell of every particle after binning against
oracle.bin_cells (the same formula, each operation rounded on its own in
plain binary64), the pair sets of the Verlet lists against
oracle.pairs_within at rc + skin, and the cover of those pairs by the
cluster-pair lists.  Pairs whose r^2 lies within the list band of
(rc + skin)^2 (a few ulps, from the halo images' rounding) may fall
either side; none occurs in these scenes at the sizes checked, but the
comparison allows them."""
import numpy as np
import pytest

from paper_2512_03565_amd import scenes
from tests import _parity as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def m():
    from paper_2512_03565_amd import mdlj
    return mdlj


def unordered(pi, pj, n):
    a = np.minimum(pi, pj).astype(np.int64)
    b = np.maximum(pi, pj).astype(np.int64)
    return a * n + b


def edge_scene():
    """SC lattice with coordinates put on cell boundaries k L / n, on 0 and L,
    just below 0 and L, and several box lengths outside the box."""
    pos, box = scenes.sc_lattice(9, 9, 10, 1.25, 0.1, seed=61)
    box = np.array([11.25, 11.25, 12.5])
    rng = np.random.default_rng(62)
    n = len(pos)
    special = []
    for L, nc in ((box[0], 4), (box[1], 4), (box[2], 5), (box[0], 3), (box[2], 4)):
        special += [k * L / nc for k in range(nc + 1)]
    special += [0.0, -0.0, -1e-300, -1e-17, 11.25 * (1 - 2.0 ** -53), 12.5 * (1 - 2.0 ** -52),
                3 * 11.25 + 0.1, -2.5 * 12.5, 1e3 + 0.3, -7e2]
    idx = rng.choice(n, (len(special), 3), replace=False)
    for (a, b, c), v in zip(idx, special):
        pos[a, 0] = v
        pos[b, 1] = v
        pos[c, 2] = v
    return pos, box


def check_cells(m, orc, pos, box, rc, skin, cfgs, label):
    # Each binning is compared with the oracle applied to that binning's
    # input: the caller's positions after set_positions, and, for a second
    # binning of the same particles, the positions the first one stored
    # (wrapped in place by x - L floor(x / L), which is checked too).  The
    # two differ only for a particle whose wrap gives exactly L: the first
    # binning clamps it into the last cell, the re-wrap of L gives 0 and the
    # first cell, the same point of the periodic box.
    n = len(pos)
    with m.System(pos, box, rc, skin=skin, precision=1) as sysm:
        for cfg in cfgs:
            sysm.set_config(cfg)
            sysm.set_positions(pos)
            r = rc if cfg[0] == m.NBR_LC else rc + skin
            stored = pos
            for rnd in range(2):
                sysm.rebuild()
                cell, nc = sysm.get_cells()
                if cfg[0] != m.NBR_VCL:
                    assert nc == tuple(orc.ncell(L, r) for L in box), (label, cfg, nc)
                ref = orc.bin_cells(stored, box, nc)
                bad = np.flatnonzero(cell != ref)
                print(f"[cells] {label} cfg={cfg} binning {rnd + 1} grid {nc}: "
                      f"{n - len(bad)}/{n} equal", flush=True)
                assert len(bad) == 0, (label, cfg, rnd, bad[:5], cell[bad[:5]], ref[bad[:5]])
                now = sysm.get_positions()
                assert np.array_equal(now, stored - box * np.floor(stored / box)), (label, cfg)
                stored = now


def vl_configs(m):
    return [(m.NBR_VL, m.ORD_I_PER_LANE, 0, 0, 0, 0), (m.NBR_VL, m.ORD_I_PER_LANE, 0, 0, 0, 1),
            (m.NBR_VL, m.ORD_WAVE_PER_I, 4, 16, 0, 0), (m.NBR_VL, m.ORD_WAVE_PER_I, 4, 16, 0, 1),
            (m.NBR_VL, m.ORD_WAVE_PER_I, 16, 4, 0, 0, 1)]


def oracle_pairs(orc, pos, box, rl):
    band = P.list_band(box, rl)
    pi, pj, r2 = orc.pairs_within(pos, box, rl * np.sqrt(1.0 + 2 * band))
    must = r2 < rl * rl * (1.0 - band)
    n = len(pos)
    return unordered(pi[must], pj[must], n), np.sort(unordered(pi, pj, n)), int((~must).sum())


def check_vl_pairs(m, orc, pos, box, rc, cfgs, label, skin=0.3, prec=1):
    n = len(pos)
    rl = rc + skin
    must, allowed, namb = oracle_pairs(orc, pos, box, rl)
    with m.System(pos, box, rc, skin=skin, precision=prec) as sysm:
        for cfg in cfgs:
            sysm.set_config(cfg)
            sysm.rebuild()
            gi, gj = sysm.get_pairs()
            n3 = cfg[5] == 1
            print(f"[vl pairs] {label} cfg={cfg}: {len(gi)} entries, oracle {len(must)} pairs "
                  f"(+{namb} in the band)", flush=True)
            assert gi.min(initial=0) >= 0 and gj.min(initial=0) >= 0, (label, cfg)
            assert gi.max(initial=0) < n and gj.max(initial=0) < n, (label, cfg)
            assert not np.any(gi == gj), (label, cfg)
            # no entry twice in a row
            directed = gi.astype(np.int64) * n + gj
            assert len(np.unique(directed)) == len(directed), (label, cfg)
            keys, counts = np.unique(unordered(gi, gj, n), return_counts=True)
            if n3:
                # Newton-3 lists: each pair once, on the smaller caller index
                assert np.all(gi < gj), (label, cfg)
                assert np.all(counts == 1), (label, cfg)
            else:
                # full lists: each pair in both directions
                assert np.all(counts == 2), (label, cfg)
            missing = np.setdiff1d(must, keys, assume_unique=True)
            extra = np.setdiff1d(keys, allowed, assume_unique=True)
            assert len(missing) == 0, (label, cfg, len(missing), missing[:5] // n, missing[:5] % n)
            assert len(extra) == 0, (label, cfg, len(extra), extra[:5] // n, extra[:5] % n)


def check_vcl_cover(m, orc, pos, box, rc, cfgs, label, skin=0.3):
    n = len(pos)
    must, _, _ = oracle_pairs(orc, pos, box, rc + skin)
    with m.System(pos, box, rc, skin=skin, precision=1) as sysm:
        for cfg in cfgs:
            sysm.set_config(cfg)
            sysm.rebuild()
            gi, gj = sysm.get_pairs()
            print(f"[vcl cover] {label} cfg={cfg}: {len(gi)} particle pairs in cluster pairs, "
                  f"oracle {len(must)}", flush=True)
            assert gj.min(initial=0) >= 0 and gi.min(initial=0) >= 0, (label, cfg)
            assert not np.any(gi == gj), (label, cfg)
            keys = np.unique(unordered(gi, gj, n))
            missing = np.setdiff1d(must, keys, assume_unique=True)
            assert len(missing) == 0, (label, cfg, len(missing))


def test_cells_config1_and_config2(m, orc):
    s = scenes.config1()
    cfgs = [(m.NBR_LC, m.ORD_I_PER_LANE, 1, 1, 0, 0), (m.NBR_VL, m.ORD_WAVE_PER_I, 16, 4, 0, 0, 1)]
    check_cells(m, orc, s["pos"], s["box"], s["rc"], 0.3, cfgs, "cfg1")
    s = scenes.config2()
    cfgs += [(m.NBR_VCL, m.ORD_CLUSTER_TILE, 4, 16, 4, 0)]
    check_cells(m, orc, s["pos"], s["box"], s["rc"], 0.3, cfgs, "cfg2")


def test_cells_on_boundaries_and_outside_the_box(m, orc):
    pos, box = edge_scene()
    cfgs = [(m.NBR_LC, m.ORD_I_PER_LANE, 1, 1, 0, 0), (m.NBR_VL, m.ORD_WAVE_PER_I, 8, 8, 0, 0),
            (m.NBR_VCL, m.ORD_I_PER_LANE, 0, 0, 8, 0)]
    check_cells(m, orc, pos, box, 2.5, 0.3, cfgs, "edges")
    # rc 3.75: cells exactly L / 3 and L / 4 wide along the axes
    check_cells(m, orc, pos, box, 3.75, 0.0, cfgs[:1], "edges rc=L/3")


def test_cells_headline_1m(m, orc):
    s = scenes.headline()
    check_cells(m, orc, s["pos"], s["box"], s["rc"], s["skin"],
                [(m.NBR_VL, m.ORD_WAVE_PER_I, 16, 4, 0, 0, 1)], "1M")


def test_vl_pairs_config1(m, orc):
    s = scenes.config1()
    check_vl_pairs(m, orc, s["pos"], s["box"], s["rc"], vl_configs(m), "cfg1")


def test_vl_pairs_config2_100k(m, orc):
    s = scenes.config2()
    check_vl_pairs(m, orc, s["pos"], s["box"], s["rc"], vl_configs(m), "cfg2")
    # the FP32-pair staged configuration builds the same list
    check_vl_pairs(m, orc, s["pos"], s["box"], s["rc"], vl_configs(m)[-1:], "cfg2 fp32", prec=0)


def test_vl_pairs_edges_sparse_and_dense(m, orc):
    pos, box = edge_scene()
    check_vl_pairs(m, orc, pos, box, 2.5, vl_configs(m), "edges")
    # cells exactly rc + skin wide: no candidate trimming by cell halves
    pos, box = scenes.fcc_lattice(16, 16, 16, 4.0 / 1.75 ** 3, 0.05, seed=43)
    check_vl_pairs(m, orc, pos, box, 2.5, vl_configs(m), "edge=rl")
    # ragged and empty cells
    box = np.array([17.0, 13.0, 11.0])
    pos = scenes.rsa_points(box, 180, 0.8, seed=63)
    check_vl_pairs(m, orc, pos, box, 2.5, vl_configs(m), "sparse")
    # neighbourhoods too large for the tiled build: the per-particle builds
    pos, box = scenes.fcc_lattice(8, 8, 8, 0.9, 0.05, seed=41)
    check_vl_pairs(m, orc, pos, box, 4.0, vl_configs(m), "dense")


def test_vl_pairs_headline_1m(m, orc):
    s = scenes.headline()
    cfgs = [(m.NBR_VL, m.ORD_WAVE_PER_I, 16, 4, 0, 0, 1), (m.NBR_VL, m.ORD_WAVE_PER_I, 4, 16, 0, 1)]
    check_vl_pairs(m, orc, s["pos"], s["box"], s["rc"], cfgs, "1M", prec=0)


def test_vcl_pairs_cover_the_list_range(m, orc):
    cfgs = [(m.NBR_VCL, m.ORD_I_PER_LANE, 0, 0, 4, 0), (m.NBR_VCL, m.ORD_CLUSTER_TILE, 4, 16, 4, 1),
            (m.NBR_VCL, m.ORD_CLUSTER_TILE, 8, 8, 8, 0), (m.NBR_VCL, m.ORD_I_PER_LANE, 0, 0, 8, 1)]
    s = scenes.config1()
    check_vcl_cover(m, orc, s["pos"], s["box"], s["rc"], cfgs, "cfg1")
    s = scenes.config4(ncell=12)
    check_vcl_cover(m, orc, s["pos"], s["box"], s["rc"], cfgs, "2-species")
    box = np.array([17.0, 13.0, 11.0])
    pos = scenes.rsa_points(box, 180, 0.8, seed=63)
    check_vcl_cover(m, orc, pos, box, 2.5, cfgs, "sparse")
    s = scenes.config2()
    check_vcl_cover(m, orc, s["pos"], s["box"], s["rc"], cfgs[:3], "cfg2")


def test_lc_has_no_pair_list(m):
    s = scenes.config1()
    with m.System(s["pos"], s["box"], s["rc"]) as sysm:
        sysm.rebuild()
        with pytest.raises(m.MdljError) as ei:
            sysm.get_pairs()
        assert ei.value.status == -2
