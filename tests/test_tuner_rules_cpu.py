"""The tuner's decision rules on scripted timing tables (no GPU): full
search reduces S samples per configuration (mean without the warm-up
sample, or minimum) and keeps the smallest, lower index on ties
(section 2.3.2); a changed particle distribution triggers a retune."""
import numpy as np
import pytest


@pytest.fixture(scope="module")
def m():
    from paper_2512_03565_amd import mdlj
    return mdlj


def test_mean_drops_warmup_and_picks_argmin(m):
    t = np.array([[900.0, 10.0, 10.0, 10.0],    # slow first sample only
                  [5.0, 12.0, 12.0, 12.0],
                  [50.0, 11.0, 11.0, 11.0]])
    vals, k = m.tune_select(t, mode=0)
    assert np.allclose(vals, [10.0, 12.0, 11.0])
    assert k == 0


def test_min_reduction(m):
    t = np.array([[9.0, 3.0, 9.0], [4.0, 4.0, 4.0]])
    vals, k = m.tune_select(t, mode=1)
    assert np.allclose(vals, [3.0, 4.0]) and k == 0


def test_ties_go_to_lower_index_and_invalid_configs_are_skipped(m):
    t = np.array([[np.inf, np.inf], [7.0, 5.0], [3.0, 5.0], [np.nan, np.nan]])
    vals, k = m.tune_select(t, mode=0)
    assert k == 1 and np.isinf(vals[0]) and np.isinf(vals[3])
    vals, k = m.tune_select(np.full((3, 2), np.inf))
    assert k == -1


def test_single_sample_is_used_as_is(m):
    vals, k = m.tune_select(np.array([[3.0], [2.0]]))
    assert np.allclose(vals, [3.0, 2.0]) and k == 1


def test_optimum_follows_a_scripted_density_change(m):
    # two phases of a run: the fastest configuration changes with density
    # (section 5: the optimal order can change during a run)
    phase1 = np.array([[10.0, 10, 10], [12.0, 12, 12], [15.0, 15, 15]])
    phase2 = np.array([[20.0, 20, 20], [14.0, 14, 14], [15.0, 15, 15]])
    assert m.tune_select(phase1)[1] == 0
    assert m.tune_select(phase2)[1] == 1


def test_retune_trigger(m):
    f0 = np.array([6.0, 0.75, 2.5, 1, 49.1, 0.10, 0.0, 1.5], np.float32)
    f1 = f0.copy()
    f1[1] *= 1.05
    assert not m.retune_needed(f0, f1, 0.1)
    f1[1] = f0[1] * 1.2
    assert m.retune_needed(f0, f1, 0.1)
    f2 = f0.copy()
    f2[5] = 0.2
    assert m.retune_needed(f0, f2, 0.1)
    # other features alone do not trigger
    f3 = f0.copy()
    f3[0] += 1
    assert not m.retune_needed(f0, f3, 0.1)
