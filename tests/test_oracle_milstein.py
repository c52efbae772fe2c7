"""Pins of the oracle's coupled Milstein scheme (the higher-order scheme of Sections 2 and 4).

* exact level means and variances of GBM under the Milstein coupling, from symbolic normal
  moments in ``milstein_closed_forms`` (a wrong Milstein constant, a wrong coarse offset 2, or
  a dropped term moves the variance by a large factor);
* order-1 strong convergence against the exact GBM solution driven by the same Brownian path,
  beside Euler-Maruyama's order 1/2 (a mis-scaled correction term loses the order);
* sigma = 0 removes both the diffusion and the correction term: Milstein equals
  Euler-Maruyama bit for bit in every precision;
* a scalar re-derivation of low-precision paths over exact rationals, rounded at every
  operation (bfloat16 and binary16 with its subnormal range);
* with Kahan compensation the rounding difference of a bfloat16 path stays much smaller.
"""

import math
from fractions import Fraction

import numpy as np
import pytest

import mlmc_workloads as W
from milstein_closed_forms import level_moments
from oracle import fp, icdf, mlmc, philox

GBM = dict(mu=0.05, sigma=0.2, x0=1.0, T=1.0, payoff=mlmc.PAYOFF_X, strike=1.0)


def _stats(r, term, m):
    return mlmc.mean_var(r["sum"][term], r["sumsq"][term], m)


@pytest.mark.parametrize("level", [0, 1, 2, 3, 4, 5])
def test_milstein_fp64_levels_match_closed_form(level):
    m = 2 ** 15
    r = mlmc.level_sums(level, m, GBM, rv_mode=mlmc.RV_EXACT, precision=fp.FP64, nested=False,
                        kahan=False, seed=21, scheme=mlmc.SCHEME_MILSTEIN)
    mean, var = _stats(r, mlmc.TERM_TWO_WAY, m)
    cf = level_moments(level)
    assert abs(mean - float(cf["mean"])) < 4.5 * math.sqrt(float(cf["var"]) / m)
    assert abs(var / float(cf["var"]) - 1) < 0.08


def test_milstein_closed_form_is_order_one():
    # the exact variances fall by a factor approaching 4 per level (strong order 1)
    v = [float(level_moments(level)["var"]) for level in range(3, 9)]
    ratios = [v[i] / v[i + 1] for i in range(len(v) - 1)]
    assert all(3.85 < q < 4.0 for q in ratios)


def _strong_mse(scheme, level, m=4096):
    paths = np.arange(m, dtype=np.uint64)
    o = mlmc.level_paths(level, paths, GBM, rv_mode=mlmc.RV_EXACT, precision=fp.FP64,
                         nested=False, kahan=False, seed=4, scheme=scheme)
    z = icdf.exact(philox.words(4, 0, level, 0, paths, 2 ** level))
    dt = 2.0 ** -level
    w_t = math.sqrt(dt) * z.sum(axis=1)
    exact = np.exp((GBM["mu"] - 0.5 * GBM["sigma"] ** 2) * 1.0 + GBM["sigma"] * w_t)
    return float(np.mean((o["Pf_hat"] - exact) ** 2))


def test_strong_order_against_exact_solution():
    levels = [3, 4, 5, 6]
    mil = [_strong_mse(mlmc.SCHEME_MILSTEIN, lv) for lv in levels]
    em = [_strong_mse(mlmc.SCHEME_EM, lv) for lv in levels]
    slope_mil = np.polyfit(levels, np.log2(mil), 1)[0]
    slope_em = np.polyfit(levels, np.log2(em), 1)[0]
    assert -2.3 < slope_mil < -1.7   # mean square error ~ delta^2
    assert -1.3 < slope_em < -0.7    # ~ delta
    assert mil[-1] < em[-1] / 20


@pytest.mark.parametrize("precision", [fp.FP64, fp.FP32, fp.FP16, fp.BF16])
@pytest.mark.parametrize("kahan", [False, True])
def test_zero_volatility_reduces_to_euler_maruyama(precision, kahan):
    sde = dict(GBM, sigma=0.0)
    kw = dict(rv_mode=mlmc.RV_CUBIC, precision=precision, nested=precision != fp.FP64,
              kahan=kahan, seed=9)
    paths = np.arange(64)
    a = mlmc.level_paths(4, paths, sde, scheme=mlmc.SCHEME_MILSTEIN, **kw)
    b = mlmc.level_paths(4, paths, sde, scheme=mlmc.SCHEME_EM, **kw)
    for key in ("Pf_bar", "Pc_bar"):
        np.testing.assert_array_equal(a[key], b[key])
    # with sigma > 0 the schemes differ
    c = mlmc.level_paths(4, paths, GBM, scheme=mlmc.SCHEME_MILSTEIN, **kw)
    d = mlmc.level_paths(4, paths, GBM, scheme=mlmc.SCHEME_EM, **kw)
    assert np.any(c["Pf_bar"] != d["Pf_bar"])


def _round(q, p, emin):
    """The rational q rounded to p significant bits, ties to even, with the subnormal
    spacing 2^(emin - p + 1) below 2^emin."""
    q = Fraction(q)
    if q == 0:
        return Fraction(0)
    e = math.floor(math.log2(abs(q)))
    while Fraction(2) ** e > abs(q):
        e -= 1
    while Fraction(2) ** (e + 1) <= abs(q):
        e += 1
    ulp = Fraction(2) ** (max(e, emin) - p + 1)
    lo = math.floor(q / ulp)
    rem = q / ulp - lo
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and lo % 2 == 1):
        lo += 1
    return lo * ulp


@pytest.mark.parametrize("precision,p,emin", [(fp.BF16, 8, -126), (fp.FP16, 11, -14), (fp.FP32, 24, -126)])
@pytest.mark.parametrize("kahan", [False, True])
def test_low_precision_paths_against_scalar_rederivation(precision, p, emin, kahan):
    level, n_paths = 2, 4
    o = mlmc.level_paths(level, np.arange(n_paths), GBM, rv_mode=mlmc.RV_CUBIC, precision=precision,
                         nested=False, kahan=kahan, seed=13, scheme=mlmc.SCHEME_MILSTEIN)
    w = philox.words(13, 0, level, 0, np.arange(n_paths, dtype=np.uint64), 2 ** level)
    z = fp.to64(icdf.approx(w, mlmc.RV_CUBIC, precision))
    R = lambda v: _round(v, p, emin)  # noqa: E731
    dt = Fraction(1, 2 ** level)
    mu, sig = 0.05, 0.2
    ca, cac = R(mu * float(dt)), R(mu * float(2 * dt))
    cb, cm = R(sig * math.sqrt(float(dt))), R(0.5 * sig * sig * float(dt))

    def step(X, c, zz, a, k):
        A = R(a * X)
        B = R(R(cb * X) * zz)
        M = R(R(cm * X) * R(R(zz * zz) - k))
        dX = R(R(A + B) + M)
        if not kahan:
            return R(X + dX), c
        y = R(dX - c)
        s = R(X + y)
        return s, R(R(s - X) - y)

    for path in range(n_paths):
        Xf = Xc = Fraction(1)
        cf = cc = Fraction(0)
        for n in range(2 ** level):
            zn = Fraction(float(z[path, n]))
            Xf, cf = step(Xf, cf, zn, ca, 1)
            if n % 2 == 1:
                zc = R(Fraction(float(z[path, n - 1])) + zn)
                Xc, cc = step(Xc, cc, zc, cac, 2)
        assert o["Pf_bar"][path] == float(Xf)
        assert o["Pc_bar"][path] == float(Xc)


def test_kahan_shrinks_milstein_rounding_difference_bf16():
    m, level = 1024, 6
    var = {}
    for kahan in (False, True):
        r = mlmc.level_sums(level, m, W.GBM, rv_mode=mlmc.RV_CUBIC, precision=fp.BF16, nested=False,
                            kahan=kahan, seed=2, diag=True, scheme=mlmc.SCHEME_MILSTEIN)
        var[kahan] = mlmc.mean_var(r["sum"][3], r["sumsq"][3], m)[1]
    rho = fp.UNIT_ROUNDOFF[fp.BF16]
    assert var[False] > 2 ** level * rho * rho / 8   # the plain path accumulates rounding error
    assert var[True] < var[False] / 8
