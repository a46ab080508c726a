"""Host logic of the tuner's training data (no GPU): merging timing sweeps
by scene index and configuration name, later files replacing earlier
timings, and the best single fixed configuration the learned tuner is
scored against (section 2.3.2's full search is the reference)."""
import numpy as np
import pytest


def _write(path, sids, names, table):
    n = len(sids)
    np.savez(path, features=np.arange(8 * n, dtype=np.float32).reshape(n, 8),
             table_us=np.asarray(table, float), names=np.array(names),
             meta=np.array([(s, 100, 0.75, 2.5, 1, 0) for s in sids], np.float64))


def test_merge_by_scene_and_name_later_file_wins(tmp_path):
    from paper_2512_03565_amd.train_tuner import load
    a = tmp_path / "a.npz"
    b = tmp_path / "b.npz"
    c = tmp_path / "c.npz"
    _write(a, [0, 1], ["x", "y", "z"], [[3.0, 2.0, 1.0], [4.0, np.inf, 6.0]])
    # a re-timing of configuration y on scene 1, and a scene only here
    _write(b, [1, 2], ["y"], [[5.0], [7.0]])
    # a re-timing that could not run (inf) keeps the earlier value
    _write(c, [0], ["x"], [[np.inf]])
    F, T, M, names = load([str(a), str(b), str(c)])
    assert names == ["x", "y", "z"]
    assert list(M[:, 0]) == [0, 1, 2]
    assert np.allclose(T[0], [3.0, 2.0, 1.0])
    assert np.allclose(T[1], [4.0, 5.0, 6.0])
    assert T[2, 1] == 7.0 and np.isinf(T[2, 0]) and np.isinf(T[2, 2])
    # features come from the first file that holds the scene
    assert np.allclose(F[1], np.arange(8, 16))


def test_best_single_configuration():
    from paper_2512_03565_amd.train_tuner import best_fixed
    t = np.array([[1.0, 1.2, 2.0],
                  [2.0, 1.0, 2.0],
                  [1.0, 1.1, np.inf]])
    k, name, g = best_fixed(t, ["a", "b", "c"])
    # c cannot run everywhere; a: (1, 2, 1) -> 2^(1/3); b: (1.2, 1, 1.1)
    assert name == "b" and k == 1
    assert g == pytest.approx((1.2 * 1.0 * 1.1) ** (1 / 3))


def test_regret_of_recorded_decisions_after_a_retiming():
    from paper_2512_03565_amd.eval_tuner import retimed_regret
    names = ["a", "b", "c"]
    table = np.array([[1.0, 2.0, 3.0],     # scene 10: a fastest
                      [2.0, 1.0, 4.0],     # scene 11: b fastest
                      [1.0, 1.5, 2.0]])    # scene 12: a fastest
    sids = [10, 11, 12]
    # c timed again: now fastest on scene 10; on 11 it could not run (inf
    # keeps the old value); scene 12 not re-timed
    retimed = (["a", "b", "c"], np.array([[np.inf, np.inf, 0.5], [np.inf, np.inf, np.inf]]),
               [10, 11])
    dec = [{"scene": 10, "chosen": "a", "fallback": False},
           {"scene": 11, "chosen": "a", "fallback": False},
           {"scene": 12, "chosen": "b", "fallback": True}]
    before, after, changed = retimed_regret(names, table, sids, retimed, dec)
    # scene 12 is not in the re-timing and is skipped
    assert changed == 1
    assert np.allclose(before, [1.0, 2.0])
    assert np.allclose(after, [2.0, 2.0])
    # a fallback ran the full search: no regret either way
    dec[1]["fallback"] = True
    before, after, _ = retimed_regret(names, table, sids, retimed, dec)
    assert np.allclose(before, [1.0, 1.0]) and np.allclose(after, [2.0, 1.0])
