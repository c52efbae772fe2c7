"""CPU tests of the host-side MLMC estimator arithmetic (Section 3)."""

import math

import pytest

from paper_2012_09739_amd import estimators as E


def test_level_stats_matches_direct_formula():
    xs = [0.5, -1.25, 3.0, 2.0, 0.125]
    s, q = sum(xs), sum(x * x for x in xs)
    mean, var = E.level_stats(s, q, len(xs))
    m = sum(xs) / 5
    assert mean == pytest.approx(m)
    assert var == pytest.approx(sum((x - m) ** 2 for x in xs) / 4)


def test_estimators():
    assert E.plain_estimate([(2.0, 4), (1.0, 2)]) == pytest.approx(1.0)
    assert E.nested_estimate([(2.0, 4), (1.0, 2)], [(0.3, 3), (-0.2, 2)]) == pytest.approx(1.0)


def test_time_models_and_speedup():
    # one level: T^ = 2 v c, T- = 2 (sqrt(v c) + sqrt(V C))^2
    assert E.time_plain([4.0], [1.0]) == pytest.approx(8.0)
    assert E.time_nested([4.0], [0.25], [0.01], [1.0]) == pytest.approx(2 * (1.0 + 0.1) ** 2)
    s = E.speedup_equal_variance([4.0], [1.0], [4.0], [0.25], [0.01], [1.0])
    assert s == pytest.approx(8.0 / (2 * 1.21))
    # the per-level bound of Section 3 dominates the actual ratio
    v_hat, c_hat = [1.0, 0.5, 0.25], [1.0, 2.0, 4.0]
    v_bar, c_bar = [1.0, 0.5, 0.25], [0.1, 0.2, 0.4]
    V_bar, C_bar = [1e-3, 5e-4, 2.5e-4], [1.2, 2.4, 4.8]
    ratio = E.time_nested(v_bar, c_bar, V_bar, C_bar) / E.time_plain(v_hat, c_hat)
    assert ratio <= max(E.per_level_factor(v_hat, c_hat, v_bar, c_bar, V_bar, C_bar)) + 1e-15


def test_optimal_samples_reach_target_variance():
    v, c, eps = [1.0, 0.3, 0.1], [1.0, 2.0, 4.0], 0.01
    m = E.optimal_samples(v, c, eps)
    assert sum(vi / mi for vi, mi in zip(v, m)) <= eps ** 2 / 2 * 1.0001
    cost = sum(mi * ci for mi, ci in zip(m, c))
    assert cost == pytest.approx(E.time_plain(v, c, eps), rel=1e-3)


def test_level_stats_needs_samples():
    with pytest.raises(ValueError):
        E.level_stats(0.0, 0.0, 0)
    assert math.isnan(E.level_stats(1.0, 1.0, 1)[1])
