"""Pins of the L2-optimal dyadic tables (Section 2.1, Figure 1, Lemmas 2.2 and 2.3).

* An independent discretisation of the same least-squares problem -- NumPy's polynomial
  least-squares fit on a dense midpoint grid of each interval with SciPy's ndtri -- gives
  the same coefficients (to the grid's quadrature error).
* Orthogonality of an L2 projection: E Z~^2 + E|Z - Z~|^2 = E Z^2 = 1 (Pythagoras, the
  fit contains the constants), checked on a regular grid of words.
* The stored table equals a fresh mpmath computation.
"""

import numpy as np
import pytest
from scipy.special import ndtri

from oracle import fp, icdf, tables


@pytest.mark.parametrize("degree", [1, 3])
def test_dense_grid_least_squares(degree):
    tab = np.array(tables.table(degree))
    n = 400000
    t = (np.arange(n) + 0.5) / n
    for j in range(1, 17):
        u = 2.0 ** -(j + 1) * (1 + t) if j < 16 else 2.0 ** -16 * t
        c = np.polynomial.polynomial.polyfit(t, ndtri(u), degree)
        tol = 1e-7 if j < 16 else 2e-4   # the log singularity of I_16 slows the midpoint rule
        np.testing.assert_allclose(c, tab[j - 1], atol=tol * (1 + np.abs(c).max()), rtol=0)


@pytest.mark.parametrize("degree,rv_mode", [(1, icdf.RV_PWL), (3, icdf.RV_CUBIC)])
def test_pythagoras_of_the_projection(degree, rv_mode):
    x = np.arange(2 ** 22, dtype=np.uint64) * np.uint64(1024) + np.uint64(511)
    z = icdf.exact(x)
    zt = icdf.approx(x, rv_mode, fp.FP64)
    lhs = np.mean(zt ** 2) + np.mean((z - zt) ** 2)
    assert abs(lhs - np.mean(z ** 2)) < 1e-6
    assert abs(np.mean(z ** 2) - 1) < 1e-3


@pytest.mark.slow
@pytest.mark.parametrize("degree", [1, 3])
def test_stored_equals_fresh(degree):
    fresh = tables.compute_table(degree)
    stored = tables.table(degree)
    np.testing.assert_array_equal(np.array(fresh), np.array(stored))


def test_piecewise_fit_is_discontinuous_like_figure_1():
    tab = np.array(tables.table(1))
    # right end of interval j+1 meets the left end of interval j: q_{j+1}(1) vs q_j(0)
    jumps = [np.polyval(tab[j][::-1], 1.0) - tab[j - 1][0] for j in range(1, 15)]
    assert all(abs(d) > 0 for d in jumps)
    assert max(abs(d) for d in jumps) < 0.05
