"""Pins of the oracle's exact and approximate inverse Gaussian CDF (Section 2.1, Section 3).

* exact: SciPy's ndtri against mpmath at 40 digits, symmetry, and Phi(Phi^{-1}(u)) = u;
* approximate: interval selection against a brute-force search over interval ends, exact
  mirror symmetry (zero mean, Assumption 2.1), boundedness, low-precision evaluation within
  its rounding bound of the float64 polynomial, the float64 evaluation against NumPy's
  polynomial routine, and E Z~^2 from exact polynomial integrals against a regular grid of
  words (a quadrature of the uniform law).
"""

import mpmath as mp
import numpy as np
import pytest
from scipy.special import ndtr

from oracle import fp, icdf, tables

rng = np.random.default_rng(7)
SPECIAL = np.array([0, 1, 2, 3, 2 ** 15, 2 ** 16 - 1, 2 ** 16, 2 ** 17, 2 ** 30, 2 ** 31 - 1,
                    2 ** 31, 2 ** 31 + 1, 2 ** 32 - 2, 2 ** 32 - 1], dtype=np.uint64)
WORDS = np.concatenate([SPECIAL, rng.integers(0, 2 ** 32, 400, dtype=np.uint64),
                        (2.0 ** rng.uniform(0, 32, 400)).astype(np.uint64)])


def test_exact_against_mpmath():
    with mp.workdps(40):
        for x in WORDS[::3]:
            u = (mp.mpf(int(x)) + mp.mpf("0.5")) / mp.mpf(2) ** 32
            ref = tables.phi_inv_mp(u)
            z = icdf.exact(x)
            assert abs(mp.mpf(float(z)) - ref) <= 1e-14 * abs(ref), int(x)


def test_exact_symmetry_and_inverse():
    z = icdf.exact(WORDS)
    zm = icdf.exact(np.uint64(2 ** 32 - 1) - WORDS)
    np.testing.assert_allclose(zm, -z, rtol=1e-14, atol=0)
    u = (WORDS.astype(np.float64) + 0.5) * 2.0 ** -32
    np.testing.assert_allclose(ndtr(z), u, rtol=1e-13)


def test_clz32_against_bit_length():
    for x in list(SPECIAL) + list(rng.integers(0, 2 ** 32, 200, dtype=np.uint64)):
        assert int(icdf.clz32(np.array([x]))[0]) == 32 - int(x).bit_length()


def test_locate_against_interval_search():
    s, j, t = icdf.locate(WORDS)
    for x, sj, jj, tt in zip(WORDS, s, j, t):
        x = int(x)
        xm = 2 ** 32 - 1 - x if x >= 2 ** 31 else x
        assert bool(sj) == (x >= 2 ** 31)
        uh = mp.mpf(xm) + mp.mpf("0.5")
        uh = uh / mp.mpf(2) ** 32                    # u' = min(u, 1 - u) exactly
        # the interval is the unique j with lower end <= u' < upper end
        ends = [mp.mpf(2) ** -(k + 1) for k in range(1, 16)]
        search = next((k for k, lo in enumerate(ends, start=1) if uh >= lo), 16)
        assert jj == search
        assert 0 <= tt < 1
        assert tables.interval_map(int(jj))(mp.mpf(float(tt))) == uh  # t is exact


@pytest.mark.parametrize("rv_mode", [icdf.RV_PWL, icdf.RV_CUBIC])
def test_approx_mirror_symmetry_is_exact(rv_mode):
    for p in (fp.FP64, fp.FP32, fp.FP16):
        z = icdf.approx(WORDS, rv_mode, p)
        zm = icdf.approx(np.uint64(2 ** 32 - 1) - WORDS, rv_mode, p)
        np.testing.assert_array_equal(zm, -z)


@pytest.mark.parametrize("rv_mode,degree", [(icdf.RV_PWL, 1), (icdf.RV_CUBIC, 3)])
def test_approx_fp64_against_numpy_polyval(rv_mode, degree):
    tab = np.array(tables.table(degree))
    s, j, t = icdf.locate(WORDS)
    want = np.array([np.polynomial.polynomial.polyval(tt, tab[jj - 1]) for jj, tt in zip(j, t)])
    want = np.where(s, -want, want)
    np.testing.assert_allclose(icdf.approx(WORDS, rv_mode, fp.FP64), want, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("rv_mode", [icdf.RV_PWL, icdf.RV_CUBIC])
@pytest.mark.parametrize("precision", [fp.FP32, fp.FP16])
def test_approx_low_precision_within_rounding_bound(rv_mode, precision):
    z64 = icdf.approx(WORDS, rv_mode, fp.FP64)
    zp = icdf.approx(WORDS, rv_mode, precision).astype(np.float64)
    rho = fp.UNIT_ROUNDOFF[precision]
    deg = 1 if rv_mode == icdf.RV_PWL else 3
    _, j, _ = icdf.locate(WORDS)
    scale = np.abs(np.array(tables.table(deg))).sum(axis=1)[j - 1]
    # coefficient, coordinate and 2d operation roundings: at most (2d + 3) rho sum|c_i|
    assert np.all(np.abs(zp - z64) <= (2 * deg + 3) * rho * scale * 1.01)
    assert np.mean(zp == z64) < 1.0 or precision == fp.FP64


@pytest.mark.parametrize("degree,rv_mode", [(1, icdf.RV_PWL), (3, icdf.RV_CUBIC)])
def test_second_moment_exact_integral_vs_word_grid(degree, rv_mode):
    tab = tables.table(degree)
    # E Z~^2 = 2 * sum_j |I_j| int_0^1 q_j(t)^2 dt  (mirror doubles the half line)
    with mp.workdps(30):
        total = mp.mpf(0)
        for j, c in enumerate(tab, start=1):
            width = mp.mpf(2) ** -(j + 1) if j < 16 else mp.mpf(2) ** -16
            sq = mp.mpf(0)
            for a, ca in enumerate(c):
                for b, cb in enumerate(c):
                    sq += mp.mpf(ca) * mp.mpf(cb) / (a + b + 1)
            total += width * sq
        exact = float(2 * total)
    # regular grid of 2^22 words: every 1024th word, offset to the middle of its block
    x = np.arange(2 ** 22, dtype=np.uint64) * np.uint64(1024) + np.uint64(511)
    grid = float(np.mean(icdf.approx(x, rv_mode, fp.FP64) ** 2))
    assert abs(grid - exact) < 2e-6
    assert 0.95 < exact < 1.0   # a variance-reducing fit: E Z~^2 < E Z^2 = 1


def test_bounded_and_cubic_more_accurate_than_linear():
    x = np.arange(2 ** 20, dtype=np.uint64) * np.uint64(4096) + np.uint64(2047)
    z = icdf.exact(x)
    e1 = np.mean((z - icdf.approx(x, icdf.RV_PWL, fp.FP64)) ** 2)
    e3 = np.mean((z - icdf.approx(x, icdf.RV_CUBIC, fp.FP64)) ** 2)
    assert e3 < e1 / 10
    for deg, mode in ((1, icdf.RV_PWL), (3, icdf.RV_CUBIC)):
        tab = np.array(tables.table(deg))
        bound = max(np.abs(tab[:, 0]).max() + np.abs(tab[:, 1:]).sum(axis=1).max(), 0)
        assert np.abs(icdf.approx(WORDS, mode, fp.FP64)).max() <= bound
