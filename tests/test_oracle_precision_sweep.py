"""Pins of the precision-width sweep in the oracle (the rounding experiments around Figure 3:
7-, 10-, 16- and 23-bit mantissas): the 17-significant-bit emulation against exact rational
arithmetic, Kahan's exact case at that width, and the rounding-difference variance
X-_N - X~_N of Lemma 2.6 across the four widths -- without compensation it scales as rho^2
(unit roundoff rho = 2^-p) and grows like N, with Kahan it is flat in N; every value below
the explicit bound B_l = N rho^2 E[X_max^2] e^{(2 mu + sigma^2) T}."""

import math
from fractions import Fraction

import numpy as np
import pytest

import mlmc_workloads as W
from oracle import fp, mlmc

WIDTHS = (fp.BF16, fp.FP16, fp.P17, fp.FP32)


def _rne(x, p):
    q = Fraction(x)
    if q == 0:
        return 0.0
    e = math.floor(math.log2(abs(q)))
    while Fraction(2) ** e > abs(q):
        e -= 1
    while Fraction(2) ** (e + 1) <= abs(q):
        e += 1
    ulp = Fraction(2) ** (e - p + 1)
    lo = math.floor(q / ulp)
    rem = q / ulp - lo
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and lo % 2 == 1):
        lo += 1
    return float(lo * ulp)


def test_p17_operations_are_correctly_rounded():
    rng = np.random.default_rng(21)
    a = fp.p17(rng.normal(size=1500) * 2.0 ** rng.integers(-20, 20, 1500))
    b = fp.p17(rng.normal(size=1500) * 2.0 ** rng.integers(-20, 20, 1500))
    assert isinstance(a + b, fp.P17Array)
    for op in (lambda u, v: u + v, lambda u, v: u - v, lambda u, v: u * v):
        got = fp.to64(op(a, b))
        want = [_rne(op(Fraction(float(u)), Fraction(float(v))), 17) for u, v in zip(fp.to64(a), fp.to64(b))]
        np.testing.assert_array_equal(got, want)
    # ties to even at 17 bits
    halves = np.array([1 + 2.0 ** -17, 1 + 3 * 2.0 ** -17])
    np.testing.assert_array_equal(fp.to64(fp.p17(halves)), [1.0, 1 + 2.0 ** -15])


def test_kahan_exact_case_p17():
    d = fp.dtype(fp.P17)
    assert float(mlmc.kahan_sum([1.0] + [2.0 ** -18] * 8, d)) == 1 + 2.0 ** -15
    naive = d(1.0)
    for _ in range(8):
        naive = naive + d(2.0 ** -18)
    assert float(naive) == 1.0


def _rounding_var(precision, level, kahan, m=1024):
    r = mlmc.level_sums(level, m, W.GBM, rv_mode=mlmc.RV_CUBIC, precision=precision, nested=False,
                        kahan=kahan, seed=2, diag=True)
    return mlmc.mean_var(r["sum"][3], r["sumsq"][3], m)[1]


def _bound(precision, level):
    N, rho = 2 ** level, fp.UNIT_ROUNDOFF[precision]
    return N * rho * rho * (1 + 0.05 / N) ** (2 * N) * math.exp(0.04) * math.exp(2 * 0.05 + 0.04)


@pytest.mark.parametrize("kahan", [False, True])
def test_rounding_variance_scales_with_unit_roundoff_squared(kahan):
    level = 5
    v = {p: _rounding_var(p, level, kahan) for p in WIDTHS}
    for p in WIDTHS:
        assert 0 < v[p] <= _bound(p, level)
    # v / rho^2 is the same constant for every width (within sampling and rounding-model noise)
    scaled = [v[p] / fp.UNIT_ROUNDOFF[p] ** 2 for p in WIDTHS]
    assert max(scaled) / min(scaled) < 2.0, scaled


def test_growth_with_N_and_flat_with_kahan_p17():
    levels = [2, 3, 4, 5, 6]
    plain = [_rounding_var(fp.P17, l, False) for l in levels]
    comp = [_rounding_var(fp.P17, l, True) for l in levels]
    slope = np.polyfit(levels, np.log2(plain), 1)[0]
    assert 0.7 < slope < 1.3
    assert max(comp) / min(comp) < 2.0
    assert comp[-1] < plain[-1] / 8
