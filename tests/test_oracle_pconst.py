"""Pins of the oracle's piecewise-constant approximate variable (a table-lookup substitute for
Z in the sense of Section 2.1): 4096 equal cells of (0, 1), value = the cell mean of Phi^{-1}.

* the stored cell means against an independent numerical quadrature of Phi^{-1} over the
  cell (SciPy quad on ndtri, and mpmath quad in the far tail), not the closed form;
* each mean lies inside its cell's range [Phi^{-1}(a), Phi^{-1}(b)] and the means increase;
* two cells (b = 1) reduce to the two-point variable +-sqrt(2/pi) = +-E|Z|;
* the word-to-cell map against a brute-force search over the cell ends in exact arithmetic;
* exact mirror symmetry (so E Z~ = 0, Assumption 2.1) in every precision;
* Z~ = E[Z | cell] makes E Z~^2 = E[Z Z~] = 1 - E|Z - Z~|^2: the table's second moment against
  the mean squared error measured over the words (far tail enumerated);
* nested binary64 level variances against the GBM closed forms with k_hb = k_bb = E Z~^2.
"""

import math
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import ndtri

from gbm_closed_forms import level_moments, word_law_mse
from oracle import fp, icdf, mlmc, tables

BITS = tables.PC_BITS
N_CELLS = 2 ** BITS
GBM = dict(mu=0.05, sigma=0.2, x0=1.0, T=1.0, payoff=mlmc.PAYOFF_X, strike=1.0)


def _means():
    return np.array(tables.pconst(), dtype=np.float64)


@pytest.mark.parametrize("i", [1, 2, 7, 100, 777, 1500, 2046, 2047])
def test_cell_means_against_quadrature(i):
    a, b = i / N_CELLS, (i + 1) / N_CELLS
    val, err = quad(ndtri, a, b, epsabs=0, epsrel=1e-13, limit=200)
    assert abs(val * N_CELLS - _means()[i]) <= 1e-12 * max(1.0, abs(_means()[i]))


def test_far_tail_cell_mean_against_mpmath_quadrature():
    # the first cell holds the logarithmic singularity of Phi^{-1} at u = 0
    with mp.workdps(30):
        f = lambda u: mp.sqrt(2) * mp.erfinv(2 * u - 1)  # noqa: E731
        pts = [mp.mpf(0)] + [mp.mpf(2) ** -e for e in (200, 100, 60, 40, 30, 20, 16, 13)] + [mp.mpf(1) / N_CELLS]
        val = mp.quad(f, pts) * N_CELLS
    assert abs(float(val) - _means()[0]) <= 1e-13 * abs(float(val))


def test_means_inside_cells_and_increasing():
    m = _means()
    edges = ndtri(np.arange(1, N_CELLS // 2 + 1) / N_CELLS)
    assert m[0] < edges[0]
    assert np.all(m[1:] > edges[:-1]) and np.all(m[1:] < edges[1:])
    assert np.all(np.diff(m) > 0) and m[-1] < 0


def test_two_cells_give_the_two_point_variable():
    (m,) = tables.compute_pconst(bits=1)
    assert m == pytest.approx(-math.sqrt(2 / math.pi), rel=1e-15)


def test_word_to_cell_map_by_brute_force():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.integers(0, 2 ** 32, 4000, dtype=np.uint64),
                        np.array([0, 1, 2 ** 20 - 1, 2 ** 20, 2 ** 31 - 1, 2 ** 31, 2 ** 32 - 1], dtype=np.uint64)])
    s, i = icdf.pconst_cell(x)
    for xv, sv, iv in zip(x.tolist(), s.tolist(), i.tolist()):
        u = Fraction(2 * xv + 1, 2 ** 33)
        um = min(u, 1 - u)
        cell = next(c for c in range(N_CELLS // 2) if Fraction(c, N_CELLS) <= um < Fraction(c + 1, N_CELLS))
        assert iv == cell and sv == (u > Fraction(1, 2))


@pytest.mark.parametrize("precision", [fp.FP64, fp.FP32, fp.FP16, fp.BF16])
def test_mirror_symmetry_and_rounding(precision):
    rng = np.random.default_rng(4)
    x = rng.integers(0, 2 ** 32, 20000, dtype=np.uint64)
    z = fp.to64(icdf.approx(x, icdf.RV_PCONST, precision))
    zm = fp.to64(icdf.approx(np.uint64(2 ** 32 - 1) - x, icdf.RV_PCONST, precision))
    np.testing.assert_array_equal(z, -zm)
    # every value is a stored mean rounded once to p
    _, i = icdf.pconst_cell(x)
    np.testing.assert_array_equal(np.abs(z), np.abs(fp.to64(fp.rn(precision, _means()[i]))))


def test_second_moment_equals_one_minus_mse():
    m = _means()
    k = 2.0 * float(np.sum(m * m)) / N_CELLS             # E Z~^2 under the uniform law
    mse = word_law_mse(icdf.exact, lambda x: icdf.approx(x, icdf.RV_PCONST, fp.FP64))
    assert 0.999 < k < 1.0
    assert abs((1.0 - k) - mse) <= 2e-3 * mse


@pytest.mark.parametrize("level", [0, 1, 3, 5])
def test_nested_fp64_levels_match_closed_form(level, m=2 ** 15):
    # The four-way variance is b^2 E|Z - Z~|^2 propagated along the path, and 89% of that
    # mean squared error sits in the two outermost cells (probability 2^-11): its sample
    # variance from 2^15 paths is not a usable estimate, so it is checked at level 0 with
    # 2^21 paths (one step) and only bounded above here.
    k = 2.0 * float(np.sum(_means() ** 2)) / N_CELLS     # E[Z Z~] = E Z~^2 for a cell mean
    cf = level_moments(level, k_hb=k, k_bb=k)
    r = mlmc.level_sums(level, m, GBM, rv_mode=mlmc.RV_PCONST, precision=fp.FP64, nested=True,
                        kahan=False, seed=15, stream=1)
    mean_a, var_a = mlmc.mean_var(r["sum"][0], r["sumsq"][0], m)
    mean_e, var_e = mlmc.mean_var(r["sum"][2], r["sumsq"][2], m)
    mean_4, var_4 = mlmc.mean_var(r["sum"][1], r["sumsq"][1], m)
    assert abs(var_a / cf["var_two_approx"] - 1) < 0.06
    assert abs(var_e / cf["var_two_exact"] - 1) < 0.06
    assert abs(mean_a - cf["mean_two"]) < 4.5 * math.sqrt(cf["var_two_approx"] / m)
    assert abs(mean_4) < 4.5 * math.sqrt(max(var_4, cf["var_four"]) / m)
    assert var_4 < 0.05 * var_e


def test_level0_four_way_variance_at_many_paths():
    m = 2 ** 21
    k = 2.0 * float(np.sum(_means() ** 2)) / N_CELLS
    cf = level_moments(0, k_hb=k, k_bb=k)
    r = mlmc.level_sums(0, m, GBM, rv_mode=mlmc.RV_PCONST, precision=fp.FP64, nested=True,
                        kahan=False, seed=16, stream=1)
    _, var_4 = mlmc.mean_var(r["sum"][1], r["sumsq"][1], m)
    assert abs(var_4 / cf["var_four"] - 1) < 0.15
