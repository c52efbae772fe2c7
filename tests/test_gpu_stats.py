"""Statistical acceptance of the packed-binary16 nested estimator at full size (2^24 paths per
level, levels 0..6, piecewise cubic on 16 dyadic intervals, binary64 exact branch).

Binary16 per-path values are compared bit for bit with the oracle elsewhere (test_gpu_parity);
here the full-size sample sets are checked against what the method fixes statistically:

* the rounding difference X-_N - X~_N (term 3: the binary16 fine state minus binary64
  arithmetic with the same approximate variables) has variance at most the explicit form
  B_l = N rho^2 E[X_max^2] e^{(2 mu + sigma^2) T} of Lemma 2.6's bound (rho = 2^-11,
  E[X_max^2] = (1 + mu delta)^{2N} e^{sigma^2}); without compensation it grows like N
  (log2-slope 1 per level), with Kahan's update (Section 2.3, Algorithm 1) it stays flat;
* the nested estimator is unbiased (Section 3): per level, the mean of the approximate
  two-way difference plus the mean of the four-way difference (independent sample sets)
  agrees with the plain binary64 two-way mean (a third independent set) by z-test;
* for P(X) = X the exact two-way part has the closed-form mean and variance of the GBM
  level difference, and the four-way difference has mean 0 in exact arithmetic (E Z~ = 0
  by the mirror, and the step is linear in Z).  With binary32 paths the rounding bias stays
  below the sampling error at 2^24 paths, so the four-way mean is 0 within 4 standard
  errors.  Binary16 paths are not unbiased: every increment A (+) B adds a constant to a
  value on the binary16 grid, and that rounding has a mean of order rho |increment| (with
  the rounded constants, about 1e-5 in X_N here, some 100 standard errors at 2^24 paths).
  The four-way term carries exactly that bias with the opposite sign, which the z-test
  above checks; at level 0 (no coarse path) the four-way mean is minus the mean of the
  rounding difference, since X^_1 - X~_1 = cb (Z - Z~) has mean 0; and the bias is bounded
  by the root of Lemma 2.6's mean-square bound (the second moment of term 3 is at most B_l).
"""

import math

import numpy as np
import pytest

import mlmc_workloads as W
from gbm_closed_forms import level_moments

import paper_2012_09739_amd as M
from paper_2012_09739_amd import estimators as E

pytestmark = pytest.mark.gpu

C3 = W.NESTED_FP16
LEVELS = C3["levels"]
N = C3["n_paths"]
RHO = 2.0 ** -11
MU, SIGMA = 0.05, 0.2
Z_MAX = 4.0


def bound_B(level):
    n = 2 ** level
    d = 2.0 ** -level
    return n * RHO ** 2 * (1 + MU * d) ** (2 * n) * math.exp(SIGMA ** 2) * math.exp(2 * MU + SIGMA ** 2)


def _run(sde, level, precision, rv_mode, kahan, stream, diag=0):
    return M.mlmc_level_run(M.level_args(sde, level, N, precision, rv_mode, kahan, C3["seed"], diag=diag,
                                         stream=stream))


def _stats(r, term):
    return E.level_stats(r["sum"][term], r["sumsq"][term], r["n_paths"])


@pytest.fixture(scope="module")
def runs():
    out = {}
    for tag, payoff in (("x", M.MLMC_PAYOFF_X), ("call", M.MLMC_PAYOFF_CALL)):
        sde = M.gbm(payoff=payoff)
        for kahan in (0, 1):
            out[tag, "nested", kahan] = [_run(sde, l, M.MLMC_FP16, M.MLMC_NESTED_CUBIC16, kahan, 1, diag=1)
                                         for l in LEVELS]
            out[tag, "approx", kahan] = [_run(sde, l, M.MLMC_FP16, M.MLMC_APPROX_CUBIC16, kahan, 0) for l in LEVELS]
        out[tag, "plain"] = [_run(sde, l, M.MLMC_FP64, M.MLMC_EXACT, 0, 2) for l in LEVELS]
    sde = M.gbm(payoff=M.MLMC_PAYOFF_X)
    for kahan in (0, 1):
        out["x", "nested32", kahan] = [_run(sde, l, M.MLMC_FP32, M.MLMC_NESTED_CUBIC16, kahan, 1, diag=1)
                                       for l in LEVELS]
    return out


def _log2_slope(levels, values):
    return float(np.polyfit(np.asarray(levels, dtype=float), np.log2(np.asarray(values)), 1)[0])


@pytest.mark.parametrize("kahan", [0, 1])
def test_rounding_variance_within_bound(runs, kahan):
    var = [_stats(r, M.MLMC_TERM_ROUNDING)[1] for r in runs["x", "nested", kahan]]
    for l, v in zip(LEVELS, var):
        assert 0 < v <= bound_B(l), (l, v, bound_B(l))
    deep = [l for l in LEVELS if l >= 2]
    slope = _log2_slope(deep, [var[l] for l in deep])
    if kahan:
        # flat in N: the compensated state keeps one rounding of the running sum
        assert abs(slope) <= 0.25, slope
        assert max(var[l] for l in deep) <= 2.0 * min(var[l] for l in deep)
    else:
        # one independent rounding per step: variance proportional to N
        assert 0.75 <= slope <= 1.25, slope


def test_kahan_reduces_rounding_variance(runs):
    plain = [_stats(r, M.MLMC_TERM_ROUNDING)[1] for r in runs["x", "nested", 0]]
    comp = [_stats(r, M.MLMC_TERM_ROUNDING)[1] for r in runs["x", "nested", 1]]
    for l in LEVELS:
        if l >= 2:
            assert comp[l] < plain[l], (l, comp[l], plain[l])
    assert comp[6] < plain[6] / 16


@pytest.mark.parametrize("payoff", ["x", "call"])
@pytest.mark.parametrize("kahan", [0, 1])
def test_nested_estimator_unbiased(runs, payoff, kahan):
    """E(P-_l - P-_{l-1}) + E(four-way) = E(P^_l - P^_{l-1}) on three independent sample sets."""
    zs = []
    tot_bar = tot_hat = tot_var = 0.0
    for l in LEVELS:
        m_a, v_a = _stats(runs[payoff, "approx", kahan][l], M.MLMC_TERM_TWO_WAY)
        m_4, v_4 = _stats(runs[payoff, "nested", kahan][l], M.MLMC_TERM_FOUR_WAY)
        m_h, v_h = _stats(runs[payoff, "plain"][l], M.MLMC_TERM_TWO_WAY)
        var = (v_a + v_4 + v_h) / N
        z = (m_a + m_4 - m_h) / math.sqrt(var)
        zs.append(z)
        tot_bar += m_a + m_4
        tot_hat += m_h
        tot_var += var
        assert abs(z) <= Z_MAX, (l, z)
    assert abs(tot_bar - tot_hat) <= Z_MAX * math.sqrt(tot_var), (tot_bar, tot_hat, zs)


@pytest.mark.parametrize("kahan", [0, 1])
def test_rounding_second_moment_within_bound(runs, kahan):
    """E|X-_N - X~_N|^2 = mean^2 + variance of term 3, within Lemma 2.6's explicit bound B_l."""
    for l, r in zip(LEVELS, runs["x", "nested", kahan]):
        m3, v3 = _stats(r, M.MLMC_TERM_ROUNDING)
        assert m3 * m3 + v3 <= bound_B(l), (l, m3, v3, bound_B(l))


@pytest.mark.parametrize("kahan", [0, 1])
def test_payoff_x_exact_pair_closed_form(runs, kahan):
    for l, r in zip(LEVELS, runs["x", "nested", kahan]):
        me, ve = _stats(r, M.MLMC_TERM_TWO_WAY_EXACT)
        want = level_moments(l)
        assert abs(me - want["mean_two"]) <= Z_MAX * math.sqrt(ve / N), (l, me, want["mean_two"])
        # relative sampling error of a variance ~ sqrt((kurtosis - 1) / N); 18 sqrt(2/N) = 6e-3
        assert abs(ve / want["var_two_exact"] - 1) <= 18 * math.sqrt(2.0 / N), (l, ve)


@pytest.mark.parametrize("kahan", [0, 1])
def test_payoff_x_four_way_mean_zero_binary32(runs, kahan):
    for l, r in zip(LEVELS, runs["x", "nested32", kahan]):
        m4, v4 = _stats(r, M.MLMC_TERM_FOUR_WAY)
        assert abs(m4) <= Z_MAX * math.sqrt(v4 / N), (l, m4, math.sqrt(v4 / N))


@pytest.mark.parametrize("kahan", [0, 1])
def test_payoff_x_four_way_bias_binary16_is_the_rounding_bias(runs, kahan):
    rs = runs["x", "nested", kahan]
    # level 0: four-way + term 3 = X^_1 - X~_1 = cb (Z - Z~), mean 0 (no coarse path)
    m4, v4 = _stats(rs[0], M.MLMC_TERM_FOUR_WAY)
    m3, v3 = _stats(rs[0], M.MLMC_TERM_ROUNDING)
    assert abs(m4 + m3) <= Z_MAX * (math.sqrt(v4 / N) + math.sqrt(v3 / N)), (m4, m3)
    # every level: the fine and the coarse path's rounding biases are each at most sqrt(B)
    for l, r in zip(LEVELS, rs):
        m4, v4 = _stats(r, M.MLMC_TERM_FOUR_WAY)
        allow = math.sqrt(bound_B(l)) + (math.sqrt(bound_B(l - 1)) if l else 0.0)
        assert abs(m4) <= allow + Z_MAX * math.sqrt(v4 / N), (l, m4, allow)
