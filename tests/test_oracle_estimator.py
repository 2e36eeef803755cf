"""Pins of the oracle's estimator arithmetic against numbers printed in the
paper (Table 4 cost formula, Sec. 5 tolerances and noise counts).  No GPU."""
import numpy as np
import pytest

from oracle import estimator


def test_cost_formula_table4():
    # Sec. 5, Example 2: eps = 0.0005 * 12^3 * 16; Table 4 variances and MVP costs
    eps = estimator.epsilon_for_volume(12 ** 3 * 16)
    assert eps == pytest.approx(13.824)
    hutch = estimator.hutchinson_cost(1.81e5, 450, eps)
    multi = estimator.cost_formula([1.37e-3, 9.56e1, 4.11e4], [825, 460, 104], eps)
    # printed 4.25e5 and 2.71e4; recomputation from the printed inputs gives
    # 4.262e5 and 2.716e4 (the inputs are themselves rounded to 3 digits)
    assert hutch == pytest.approx(4.26e5, rel=2e-3)
    assert multi == pytest.approx(2.716e4, rel=2e-3)
    assert abs(hutch / 4.25e5 - 1) < 0.01 and abs(multi / 2.71e4 - 1) < 0.01


def test_noise_count_sums_tables():
    assert 2 + 138 + 2367 == 2507
    assert 2 + 1107 + 1815 == 2924
    assert 2 + 6 + 276 == 284


def test_level_tolerances():
    eps = 10.0
    t1, t2, t3 = estimator.level_tolerances(eps, [3.0, 4.0])
    assert t1 == pytest.approx(eps / np.sqrt(3))
    assert t2 == pytest.approx(np.sqrt(100 - 9) / np.sqrt(2))
    assert t3 == pytest.approx(np.sqrt(100 - 25))
    # if every level meets its target the combined error meets eps
    e1 = t1
    e2 = estimator.level_tolerances(eps, [e1])[1]
    e3 = estimator.level_tolerances(eps, [e1, e2])[2]
    assert np.sqrt(e1 ** 2 + e2 ** 2 + e3 ** 2) == pytest.approx(eps)


def test_check_points():
    assert estimator.check_points(1, 5) == [2, 3, 4, 5]
    assert estimator.check_points(2, 12) == [3, 6, 9, 12]
    assert estimator.check_points(3, 15) == [6, 9, 12, 15]


def test_level_estimate_stats():
    s = np.array([1 + 1j, 2 - 1j, 3 + 0j, 6 + 2j])
    est = estimator.level_estimate(s, c=np.array([0.5, 0.25j]))
    assert est.mean == pytest.approx(3 + 0.5j)
    assert est.var == pytest.approx(np.sum(np.abs(s - s.mean()) ** 2) / 3)
    assert est.stderr == pytest.approx(np.sqrt(est.var / 4))
    assert est.estimate == pytest.approx(3.5 + 0.75j)
