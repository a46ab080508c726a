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


# ------------------------------------------------------- early-stopping search

def _table():
    # [K, S]: sample 0 = warm-up cycle, samples 1..3 timed cycles
    return np.array([[20.0, 10.0, 10.0, 10.0],   # the best
                     [18.0, 25.0, 25.0, 25.0],   # warm-up within 2x, first cycle far off
                     [90.0, 50.0, 50.0, 50.0],   # warm-up beyond 2x the best
                     [19.0, 10.5, 10.4, 10.6],   # close to the best: measured in full
                     [np.inf, np.inf, np.inf, np.inf]])  # cannot run


def test_early_stop_best_first_drops_the_rest(m):
    vals, taken, k = m.tune_select_early(_table())
    assert k == 0
    # 0 and 3 measured in full, 1 dropped after its first timed cycle, 2 after
    # its warm-up, 4 after its (infinite) first sample
    assert list(taken) == [4, 2, 1, 4, 1]
    assert vals[0] == pytest.approx(10.0) and vals[3] == pytest.approx(10.5)
    assert vals[1] == 25.0 and vals[2] == 90.0 and np.isinf(vals[4])


def test_early_stop_equals_full_search_when_nothing_is_dropped(m):
    t = _table()
    full_vals, full_k = m.tune_select(t, mode=0)
    # a generous margin keeps every runnable configuration
    vals, taken, k = m.tune_select_early(t, warm_factor=1e9, margin=1e9)
    assert k == full_k
    assert np.allclose(vals[:4], full_vals[:4])
    assert list(taken[:4]) == [4, 4, 4, 4]


def test_early_stop_order_changes_cost_not_choice(m):
    t = _table()
    # the best visited last: everything before it is measured in full
    vals, taken, k = m.tune_select_early(t, order=[2, 1, 3, 4, 0])
    assert k == 0
    assert taken[2] == 4 and taken[1] == 4 and taken[3] == 4
    # the best visited first: fewer samples in total
    _, taken_first, k_first = m.tune_select_early(t, order=[0, 3, 1, 2, 4])
    assert k_first == 0 and taken_first.sum() < taken.sum()


def test_early_stop_can_miss_a_configuration_with_a_slow_warmup(m):
    # a configuration whose warm-up cycle (which includes the structure
    # build) is slow but whose steps are fastest is dropped once a good one
    # has been measured: the price of stopping early
    t = np.array([[20.0, 10.0, 10.0, 10.0],
                  [45.0, 8.0, 8.0, 8.0]])
    assert m.tune_select(t)[1] == 1
    vals, taken, k = m.tune_select_early(t)
    assert k == 0 and list(taken) == [4, 1]


def test_early_stop_ties_and_bad_arguments(m):
    t = np.array([[5.0, 3.0, 3.0], [5.0, 3.0, 3.0]])
    assert m.tune_select_early(t, order=[1, 0])[2] == 0
    with pytest.raises(m.MdljError):
        m.tune_select_early(t, order=[0, 0])
    with pytest.raises(m.MdljError):
        m.tune_select_early(t, warm_factor=0.5)


# ------------------------------------------------------- energy as the metric

def test_energy_optimum_can_differ_from_time_optimum(m):
    # section 2.3.3: tuning for energy instead of runtime.  Energy per step
    # is power times time: the fastest configuration draws the most power
    us = np.array([100.0, 110.0, 140.0, np.inf])
    watts = np.array([900.0, 700.0, 600.0, 500.0])
    uj, k = m.tune_select_energy(us, watts)
    assert np.allclose(uj[:3], [90000.0, 77000.0, 84000.0]) and np.isinf(uj[3])
    assert k == 1
    assert m.tune_select(us[:, None])[1] == 0


def test_energy_rule_ties_and_invalid(m):
    uj, k = m.tune_select_energy([2.0, 1.0, 4.0], [1.0, 2.0, 0.5])
    assert k == 0 and np.allclose(uj, [2.0, 2.0, 2.0])
    uj, k = m.tune_select_energy([np.nan, 1.0], [1.0, -3.0])
    assert k == -1 and np.all(np.isinf(uj))
