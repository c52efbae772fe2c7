"""Pins of the oracle's coupled Euler-Maruyama levels, Kahan updates and MLMC differences.

Pins used (none re-types the oracle's own formula):
* GBM closed forms (exact moment recursions in ``gbm_closed_forms``): level means and
  variances of the exact and approximate two-way differences and of the four-way
  difference; a coupling mistake (wrong pairing, wrong coarse constant, unshared
  uniforms) moves a variance by orders of magnitude;
* the call payoff at level 0 in closed form;
* telescoping of the level means (Section 3);
* per-path identity four-way = exact two-way - approximate two-way;
* exact rational arithmetic on tiny inputs: the oracle's float path stays within the
  standard-model rounding bound of the exactly computed path;
* Kahan exact cases and the Kahan error bound (Section 2.3);
* Lemma 2.4 by enumeration over a regular grid of words; Lemma 2.6 slope of the
  rounding-difference variance and its explicit bound.
"""

import math
from fractions import Fraction

import numpy as np
import pytest

from gbm_closed_forms import call_level0_mean, level_moments, table_second_moment, word_law_mse
from oracle import fp, icdf, mlmc, philox, tables

GBM = dict(mu=0.05, sigma=0.2, x0=1.0, T=1.0, payoff=mlmc.PAYOFF_X, strike=1.0)


def _kappa(rv_mode):
    """(E[Z Z~], E[Z~^2]) under the law of the 32-bit words: E Z~^2 is the exact table
    integral and E[Z Z~] is fixed by E|Z - Z~|^2 over the words (far tail enumerated), so
    that the four-way combination 1 - 2 E[Z Z~] + E Z~^2 equals that mean squared error."""
    k_bb = table_second_moment(tables.table(1 if rv_mode == mlmc.RV_PWL else 3))
    mse = word_law_mse(icdf.exact, lambda x: icdf.approx(x, rv_mode, fp.FP64))
    return (1.0 + k_bb - mse) / 2, k_bb


def _stats(r, term, m):
    return mlmc.mean_var(r["sum"][term], r["sumsq"][term], m)


@pytest.mark.parametrize("level", [0, 1, 2, 3, 4, 5])
def test_plain_fp64_levels_match_closed_form(level):
    m = 2 ** 15
    r = mlmc.level_sums(level, m, GBM, rv_mode=mlmc.RV_EXACT, precision=fp.FP64,
                        nested=False, kahan=False, seed=11)
    mean, var = _stats(r, mlmc.TERM_TWO_WAY, m)
    cf = level_moments(level)
    assert abs(mean - cf["mean_two"]) < 4.5 * math.sqrt(cf["var_two_exact"] / m)
    assert abs(var / cf["var_two_exact"] - 1) < 0.06


@pytest.mark.parametrize("level", [0, 1, 3, 5])
def test_nested_fp64_levels_match_closed_form(level, rv_mode=mlmc.RV_PWL, m=2 ** 15):
    # Piecewise linear only: the cubic fit's squared error sits 85% in the far-tail
    # interval I_16 and is dominated there by words of probability ~2^-30, so a sample
    # variance of its four-way difference is not a usable estimate at any test size.
    k_hb, k_bb = _kappa(rv_mode)
    cf = level_moments(level, k_hb=k_hb, k_bb=k_bb)
    r = mlmc.level_sums(level, m, GBM, rv_mode=rv_mode, precision=fp.FP64, nested=True,
                        kahan=False, seed=5, stream=1)
    mean_a, var_a = _stats(r, mlmc.TERM_TWO_WAY, m)
    mean_4, var_4 = _stats(r, mlmc.TERM_FOUR_WAY, m)
    mean_e, var_e = _stats(r, mlmc.TERM_TWO_WAY_EXACT, m)
    assert abs(var_a / cf["var_two_approx"] - 1) < 0.06
    assert abs(var_e / cf["var_two_exact"] - 1) < 0.06
    assert abs(var_4 / cf["var_four"] - 1) < 0.15
    assert abs(mean_4) < 4.5 * math.sqrt(cf["var_four"] / m)
    assert abs(mean_a - cf["mean_two"]) < 4.5 * math.sqrt(cf["var_two_approx"] / m)
    # the four-way difference is much smaller than either two-way difference
    assert var_4 < 0.1 * var_e


def test_call_payoff_level0_closed_form():
    m = 2 ** 16
    sde = dict(GBM, payoff=mlmc.PAYOFF_CALL)
    r = mlmc.level_sums(0, m, sde, rv_mode=mlmc.RV_EXACT, precision=fp.FP64, nested=False,
                        kahan=False, seed=3)
    mean, var = _stats(r, 0, m)
    assert abs(mean - call_level0_mean()) < 4.5 * math.sqrt(var / m)


def test_telescoping_sum_of_levels():
    L, m = 5, 2 ** 14
    total, se2 = 0.0, 0.0
    for level in range(L + 1):
        r = mlmc.level_sums(level, m, GBM, rv_mode=mlmc.RV_EXACT, precision=fp.FP64,
                            nested=False, kahan=False, seed=100 + level)
        mean, var = _stats(r, 0, m)
        total += mean
        se2 += var / m
    target = (1 + 0.05 * 2.0 ** -L) ** (2 ** L)       # E[P^_L] of the finest level
    assert abs(sum(level_moments(l)["mean_two"] for l in range(L + 1)) - target) < 1e-12
    assert abs(total - target) < 4.5 * math.sqrt(se2)


@pytest.mark.parametrize("precision", [fp.FP32, fp.FP16])
def test_four_way_identity_per_path(precision):
    r = mlmc.level_paths(4, np.arange(500), dict(GBM, payoff=mlmc.PAYOFF_CALL),
                         rv_mode=mlmc.RV_PWL, precision=precision, nested=True, kahan=True,
                         seed=9, stream=1, diag=True)
    t = r["terms"]
    np.testing.assert_allclose(t[1] + t[0], t[2], rtol=0, atol=4e-16)
    np.testing.assert_array_equal(t[2], r["Pf_hat"] - r["Pc_hat"])
    assert not np.any(np.isnan(t))


def _exact_path(level, z_values, ca_f, ca_c, cb, x0):
    """Fine and coarse states in exact rational arithmetic from given (rounded) inputs."""
    Xf, Xc = Fraction(x0), Fraction(x0)
    ca_f, ca_c, cb = Fraction(ca_f), Fraction(ca_c), Fraction(cb)
    zs = [Fraction(z) for z in z_values]
    for n, z in enumerate(zs):
        Xf = Xf + ca_f * Xf + cb * Xf * z
        if level >= 1 and n % 2 == 1:
            Xc = Xc + ca_c * Xc + cb * Xc * (zs[n - 1] + z)
    return Xf, Xc


@pytest.mark.parametrize("precision,kahan", [(fp.FP64, False), (fp.FP32, False),
                                             (fp.FP32, True), (fp.FP16, False), (fp.FP16, True)])
def test_paths_within_rounding_bound_of_exact_arithmetic(precision, kahan):
    level, paths = 4, np.arange(6)
    mode = mlmc.RV_EXACT if precision == fp.FP64 else mlmc.RV_PWL
    r = mlmc.level_paths(level, paths, GBM, rv_mode=mode, precision=precision, nested=False,
                         kahan=kahan, seed=21)
    w = philox.words(21, 0, level, 0, paths, 2 ** level)
    ca_f, ca_c, cb, x0, _, _ = mlmc.constants(GBM, level, precision)
    rho = fp.UNIT_ROUNDOFF[precision]
    N = 2 ** level
    key_f, key_c = ("Pf_hat", "Pc_hat") if precision == fp.FP64 else ("Pf_bar", "Pc_bar")
    for i in range(paths.size):
        if precision == fp.FP64:
            z = icdf.exact(w[i])
            zc_round = None
        else:
            z = icdf.approx(w[i], mlmc.RV_PWL, precision)
            # the coarse path consumes the rounded pairwise sums
            zc_round = [z[n - 1] + z[n] for n in range(1, N, 2)]
        Xf, Xc = _exact_path(level, [float(v) for v in z], float(ca_f), float(ca_c), float(cb), float(x0))
        if zc_round is not None:
            Xc = Fraction(float(x0))
            for zc in zc_round:
                Xc = Xc + Fraction(float(ca_c)) * Xc + Fraction(float(cb)) * Xc * Fraction(float(zc))
        # standard model: each step adds at most ~4 rho |X| of error; N steps
        assert abs(Fraction(r[key_f][i]) - Xf) <= 5 * N * rho * 1.2
        assert abs(Fraction(r[key_c][i]) - Xc) <= 5 * N * rho * 1.2
        # and the path is far from the exact one only by rounding: a dropped or
        # mis-indexed term would move it by O(sqrt(delta))
        assert abs(float(Xf) - 1.0) < 1.0


def test_kahan_exact_cases():
    h = np.float16
    assert mlmc.kahan_sum([1.0] + [2.0 ** -12] * 8, h) == h(1 + 2.0 ** -9)
    naive = h(1.0)
    for _ in range(8):
        naive = naive + h(2.0 ** -12)
    assert naive == h(1.0)
    s = np.float32
    assert mlmc.kahan_sum([1.0] + [2.0 ** -25] * 16, s) == s(1 + 2.0 ** -21)
    xs = [1.0] + [2.0 ** -54] * 4                  # exact sum 1 + 2^-52 is representable
    assert mlmc.kahan_sum(xs, np.float64) == 1.0 + 2.0 ** -52
    assert math.fsum(xs) == 1.0 + 2.0 ** -52 and sum(xs) == 1.0


@pytest.mark.parametrize("dtype,rho", [(np.float32, 2.0 ** -24), (np.float16, 2.0 ** -11)])
def test_kahan_error_bound(dtype, rho):
    rng = np.random.default_rng(3)
    for trial in range(20):
        n = 200
        xs = (rng.normal(0.01, 0.1, n)).astype(dtype)
        xs[0] = dtype(1.0)
        exact = math.fsum(float(v) for v in xs)
        got = float(mlmc.kahan_sum(xs, dtype))
        bound = (2 * rho + n * rho * rho) * sum(abs(float(v)) for v in xs)
        assert abs(got - exact) <= bound


def test_lemma_2_4_rounding_error_of_state_update_has_tiny_mean():
    """eta = (X (+) R(beta)) - (X + R(beta)) over all words of a regular grid."""
    level = 6
    ca_f, _, cb, _, _, _ = mlmc.constants(GBM, level, fp.FP16)
    X = np.float16(1.2345)
    x = np.arange(2 ** 22, dtype=np.uint64) * np.uint64(1024) + np.uint64(511)
    Zt = icdf.approx(x, mlmc.RV_CUBIC, fp.FP16)
    dX = ca_f * X + (cb * X) * Zt
    eta = (X + dX).astype(np.float64) - (np.float64(X) + dX.astype(np.float64))
    rho = fp.UNIT_ROUNDOFF[fp.FP16]
    mean_abs = np.mean(np.abs(eta))
    assert 0.2 * rho < mean_abs < 2 * rho          # E|eta| = O(rho)
    assert abs(np.mean(eta)) < 0.05 * mean_abs      # E(eta) = O(rho^2) << E|eta|


def test_lemma_2_6_rounding_difference_growth_and_bound():
    m = 2048
    var_plain, var_kahan = [], []
    for level in range(2, 7):
        for kahan, store in ((False, var_plain), (True, var_kahan)):
            r = mlmc.level_sums(level, m, GBM, rv_mode=mlmc.RV_CUBIC, precision=fp.FP16,
                                nested=False, kahan=kahan, seed=1, diag=True)
            store.append(_stats(r, mlmc.TERM_ROUNDING, m)[1])
        N = 2 ** level
        rho = fp.UNIT_ROUNDOFF[fp.FP16]
        dt = 2.0 ** -level
        ex2_max = (1 + 0.05 * dt) ** (2 * N) * math.exp(0.04)
        bound = N * rho * rho * ex2_max * math.exp(2 * 0.05 + 0.04)
        assert var_plain[-1] <= bound
        assert var_kahan[-1] <= bound
    slope_plain = np.polyfit(range(2, 7), np.log2(var_plain), 1)[0]
    slope_kahan = np.polyfit(range(2, 7), np.log2(var_kahan), 1)[0]
    assert 0.6 < slope_plain < 1.4      # Var grows like N (Lemma 2.6)
    assert slope_kahan < 0.5            # compensated: roughly flat in N (Section 2.3)
    assert var_kahan[-1] < var_plain[-1] / 4
