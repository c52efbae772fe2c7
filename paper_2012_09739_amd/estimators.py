"""MLMC estimator arithmetic on the host (Section 3): level statistics, the plain and nested
estimators, optimal sample allocation, total-time models and the equal-variance speed-up.

All inputs are the per-level sums, sums of squares, sample counts and device costs the
C-ABI returns; nothing here touches the GPU.

* plain estimator   theta^ = sum_l (1/m^_l) sum (P^_l - P^_{l-1})
* nested estimator  theta- = sum_l (1/m-_l) sum (P-_l - P-_{l-1})
                              + (1/M-_l) sum (P^_l - P^_{l-1} - P-_l + P-_{l-1})
* times to reach mean squared error eps^2 (optimal allocation m_l ~ sqrt(v_l / c_l)):
    T^ = 2 eps^-2 (sum_l sqrt(v^_l c^_l))^2
    T- = 2 eps^-2 (sum_l sqrt(v-_l c-_l) + sqrt(V-_l C-_l))^2
  so the speed-up at equal total MLMC variance, T^ / T-, does not depend on eps.
* per-level bound  T- <= T^ max_l { (v-_l c-_l)/(v^_l c^_l) (1 + sqrt(V-_l C-_l / (v-_l c-_l)))^2 }
"""

import math


def level_stats(total, total_sq, m):
    """(mean, unbiased variance) of one term from its sum and sum of squares over m samples."""
    if m < 1:
        raise ValueError("need at least one sample")
    mean = total / m
    if m == 1:
        return mean, math.nan
    var = (total_sq - total * total / m) / (m - 1)
    return mean, max(var, 0.0)


def plain_estimate(level_sums):
    """theta^ from [(sum, m), ...] of the two-way differences of levels 0..L."""
    return math.fsum(s / m for s, m in level_sums)


def nested_estimate(two_way_sums, four_way_sums):
    """theta- from [(sum, m-_l)] of the approximate two-way and [(sum, M-_l)] of the four-way."""
    if len(two_way_sums) != len(four_way_sums):
        raise ValueError("one entry per level for both terms")
    return math.fsum([s / m for s, m in two_way_sums] + [s / m for s, m in four_way_sums])


def optimal_samples(v, c, eps):
    """m_l = ceil(2 eps^-2 sqrt(v_l / c_l) sum_k sqrt(v_k c_k)), the allocation behind T."""
    total = math.fsum(math.sqrt(vi * ci) for vi, ci in zip(v, c))
    return [max(1, math.ceil(2.0 / eps ** 2 * math.sqrt(vi / ci) * total)) for vi, ci in zip(v, c)]


def time_plain(v_hat, c_hat, eps=1.0):
    return 2.0 / eps ** 2 * math.fsum(math.sqrt(v * c) for v, c in zip(v_hat, c_hat)) ** 2


def time_nested(v_bar, c_bar, V_bar, C_bar, eps=1.0):
    return 2.0 / eps ** 2 * math.fsum(math.sqrt(v * c) + math.sqrt(V * C)
                                      for v, c, V, C in zip(v_bar, c_bar, V_bar, C_bar)) ** 2


def speedup_equal_variance(v_hat, c_hat, v_bar, c_bar, V_bar, C_bar):
    """T^ / T- (independent of the target accuracy)."""
    return time_plain(v_hat, c_hat) / time_nested(v_bar, c_bar, V_bar, C_bar)


def per_level_factor(v_hat, c_hat, v_bar, c_bar, V_bar, C_bar):
    """The per-level factors whose maximum bounds T- / T^ (and their reciprocals are the
    per-level speed-ups)."""
    out = []
    for vh, ch, vb, cb, VB, CB in zip(v_hat, c_hat, v_bar, c_bar, V_bar, C_bar):
        out.append((vb * cb) / (vh * ch) * (1.0 + math.sqrt((VB * CB) / (vb * cb))) ** 2)
    return out
