"""Pins of the oracle's bfloat16 emulation (8 significant bits, round to nearest even): the
rounding function against IEEE conversions NumPy performs itself (p = 24 and p = 11) and
against exact rational arithmetic (p = 8), correctly rounded + - x, the Kahan exact case of
Section 2.3 at this precision, Kahan's error bound, and Lemma 2.6's growth of the rounding
difference with N (flat with compensation) under the explicit bound with rho = 2^-8."""

import math
from fractions import Fraction

import numpy as np
import pytest

import mlmc_workloads as W
from oracle import fp, mlmc


def _rne_fraction(x, p):
    """x rounded to p significant bits from its exact rational value (brute force)."""
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


def test_round_bits_matches_ieee_conversions():
    rng = np.random.default_rng(11)
    x = rng.normal(size=200000) * 10.0 ** rng.integers(-4, 4, 200000)
    np.testing.assert_array_equal(fp.round_bits(x, 24), x.astype(np.float32).astype(np.float64))
    normal16 = np.abs(x) >= 2.0 ** -14
    np.testing.assert_array_equal(fp.round_bits(x[normal16], 11),
                                  x[normal16].astype(np.float16).astype(np.float64))


def test_round_bits_against_exact_rationals():
    rng = np.random.default_rng(12)
    x = rng.normal(size=3000) * 10.0 ** rng.integers(-6, 6, 3000)
    # values exactly halfway between neighbours at 8 bits, both parities
    x = np.concatenate([x, [1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(3 + 2.0 ** -7), 255.5, 254.5]])
    got = fp.round_bits(x, 8)
    want = np.array([_rne_fraction(float(v), 8) for v in x])
    np.testing.assert_array_equal(got, want)


def test_bf16_operations_are_correctly_rounded():
    rng = np.random.default_rng(13)
    a = fp.bf16(rng.normal(size=2000) * 2.0 ** rng.integers(-12, 12, 2000))
    b = fp.bf16(rng.normal(size=2000) * 2.0 ** rng.integers(-12, 12, 2000))
    for op in (lambda u, v: u + v, lambda u, v: u - v, lambda u, v: u * v):
        got = fp.to64(op(a, b))
        want = [_rne_fraction(float(op(Fraction(float(u)), Fraction(float(v)))), 8)
                for u, v in zip(fp.to64(a), fp.to64(b))]
        np.testing.assert_array_equal(got, want)


def test_kahan_exact_case_bf16():
    b = fp.dtype(fp.BF16)
    assert float(mlmc.kahan_sum([1.0] + [2.0 ** -9] * 8, b)) == 1 + 2.0 ** -6
    naive = b(1.0)
    for _ in range(8):
        naive = naive + b(2.0 ** -9)
    assert float(naive) == 1.0


def test_kahan_error_bound_bf16():
    rho = fp.UNIT_ROUNDOFF[fp.BF16]
    rng = np.random.default_rng(14)
    for _ in range(20):
        n = 200
        xs = fp.to64(fp.bf16(rng.normal(0.01, 0.1, n)))
        xs[0] = 1.0
        exact = math.fsum(xs.tolist())
        got = float(mlmc.kahan_sum(xs.tolist(), fp.dtype(fp.BF16)))
        assert abs(got - exact) <= (2 * rho + n * rho * rho) * float(np.abs(xs).sum())


def test_lemma_2_6_rounding_difference_bf16():
    m = 1024
    var_plain, var_kahan = [], []
    for level in range(2, 6):
        for kahan, store in ((False, var_plain), (True, var_kahan)):
            r = mlmc.level_sums(level, m, W.GBM, rv_mode=mlmc.RV_CUBIC, precision=fp.BF16,
                                nested=False, kahan=kahan, seed=2, diag=True)
            store.append(mlmc.mean_var(r["sum"][3], r["sumsq"][3], m)[1])
        N = 2 ** level
        rho = fp.UNIT_ROUNDOFF[fp.BF16]
        dt = 2.0 ** -level
        bound = N * rho * rho * (1 + 0.05 * dt) ** (2 * N) * math.exp(0.04) * math.exp(2 * 0.05 + 0.04)
        assert var_plain[-1] <= bound and var_kahan[-1] <= bound
    slope_plain = np.polyfit(range(2, 6), np.log2(var_plain), 1)[0]
    assert 0.6 < slope_plain < 1.4
    assert var_kahan[-1] < var_plain[-1] / 4


@pytest.mark.parametrize("kahan", [False, True])
def test_bf16_paths_against_scalar_rederivation(kahan):
    """Two paths of level 2 by a scalar loop over exact rationals rounded at every step."""
    level, sde = 2, W.GBM
    o = mlmc.level_paths(level, np.arange(2), sde, rv_mode=mlmc.RV_PWL, precision=fp.BF16, nested=False,
                         kahan=kahan, seed=7)
    from oracle import icdf, philox
    w = philox.words(7, 0, level, 0, np.arange(2, dtype=np.uint64), 4)
    z = fp.to64(icdf.approx(w, mlmc.RV_PWL, fp.BF16))
    R = lambda v: _rne_fraction(float(v), 8)  # noqa: E731
    dt = 2.0 ** -level
    ca, cb = R(0.05 * dt), R(0.2 * math.sqrt(dt))
    for p in range(2):
        X, c = 1.0, 0.0
        for n in range(4):
            A = R(Fraction(ca) * Fraction(X))
            B = R(Fraction(R(Fraction(cb) * Fraction(X))) * Fraction(z[p, n]))
            dX = R(Fraction(A) + Fraction(B))
            if kahan:
                y = R(Fraction(dX) - Fraction(c))
                s = R(Fraction(X) + Fraction(y))
                c = R(Fraction(R(Fraction(s) - Fraction(X))) - Fraction(y))
                X = s
            else:
                X = R(Fraction(X) + Fraction(dX))
        assert o["Pf_bar"][p] == X
