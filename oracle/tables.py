"""Piecewise-polynomial approximations of the inverse Gaussian CDF on dyadic intervals.

Test infrastructure only.  Section 2.1 replaces Phi^{-1} by a piecewise polynomial
Phi~^{-1} (piecewise linear, Lemma 2.2 and Figure 1; piecewise cubic, Lemma 2.3), built on
intervals that shrink geometrically towards the tails, and defers the construction to the
authors' companion work.  The reading used throughout this repository (stated because the
paper is silent on it):

* 16 intervals of (0, 1/2]:  I_j = [2^-(j+1), 2^-j) for j = 1..15 and I_16 = (0, 2^-16);
  (1/2, 1) is covered by mirror symmetry, Phi~^{-1}(1-u) = -Phi~^{-1}(u), which makes the
  approximate variable exactly zero-mean (Assumption 2.1).
* On each interval an independent polynomial of degree d (1: linear, 3: cubic) in the
  local coordinate t in [0, 1) -- u = 2^-(j+1) (1 + t) on I_1..I_15 and u = 2^-16 t on
  I_16 -- chosen to minimise the L2 error  int_0^1 (Phi^{-1}(u(t)) - q_j(t))^2 dt, i.e.
  the mean squared error E|Z - Z~|^2 under the uniform law of U restricted to I_j.
  Independent fits are discontinuous at interval ends, which produces the tiny
  zero-measure gaps in the density that Figure 1(b) shows.

The fit is the least-squares normal equations  H c = m  with the Hilbert matrix
H_ik = 1/(i+k+1) and moments m_i = int_0^1 Phi^{-1}(u(t)) t^i dt, evaluated with mpmath
(tanh-sinh quadrature handles the logarithmic singularity of I_16 at t = 0).

Pinned by ``tests/test_oracle_tables.py``: a dense-grid weighted least-squares fit with
NumPy (an independent discretisation of the same minimisation) reproduces the
coefficients, the residual is orthogonal to 1, t, ..., t^d, and the stored table equals a
fresh computation.

A further approximate variable (Section 2.1 names table lookups and the Rademacher
variables of the weak Euler-Maruyama scheme among the substitutes for Z): the
piecewise-constant inverse CDF on 2^b equal cells of (0, 1), cell i = [i 2^-b, (i+1) 2^-b),
whose value is the cell mean of Phi^{-1} -- the L2-optimal constant, i.e. Z~ = E[Z | cell]:

    mean_i = 2^b int_a^b' Phi^{-1}(u) du = 2^b (phi(Phi^{-1}(a)) - phi(Phi^{-1}(b')))

(substitute u = Phi(z): int z phi(z) dz = -phi(z)).  Only the lower half (i < 2^(b-1)) is
stored; the upper half is its mirror.  b = 1 gives the two-point variable +-sqrt(2/pi).
Pinned by ``tests/test_oracle_pconst.py``.
"""

import functools
import json
import os

import mpmath as mp

N_INTERVALS = 16
DEGREES = {"pwl": 1, "cubic": 3}
_STORED = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "tests", "golden", "dyadic_tables.json")


def phi_inv_mp(u):
    """Phi^{-1}(u) = sqrt(2) erfinv(2u - 1) in mpmath, with working precision raised so
    that 2u - 1 keeps all digits of a tiny u."""
    u = mp.mpf(u)
    extra = int(-mp.log10(u)) + 10 if u < mp.mpf("0.25") else 0
    with mp.workdps(mp.mp.dps + extra):
        return mp.sqrt(2) * mp.erfinv(2 * u - 1)


def interval_map(j):
    """u(t) for the local coordinate t in [0, 1) of interval j (1-based)."""
    if not 1 <= j <= N_INTERVALS:
        raise ValueError("interval index out of range")
    if j < N_INTERVALS:
        lo = mp.mpf(2) ** (-(j + 1))
        return lambda t: lo * (1 + t)
    scale = mp.mpf(2) ** (-N_INTERVALS)
    return lambda t: scale * t


def _moments(j, degree):
    u_of_t = interval_map(j)
    f = lambda t: phi_inv_mp(u_of_t(t))  # noqa: E731
    # split the singular interval geometrically towards t = 0 so tanh-sinh converges fast
    pts = [0] + [mp.mpf(2) ** (-e) for e in (60, 40, 20, 10, 5)] + [1] if j == N_INTERVALS else [0, 1]
    return [mp.quad(lambda t, i=i: f(t) * t ** i, pts) for i in range(degree + 1)]


def fit_interval(j, degree, dps=30):
    """L2-optimal monomial coefficients c_0..c_d (in t) on interval j, as mpf."""
    with mp.workdps(dps):
        m = _moments(j, degree)
        hilbert = mp.matrix(degree + 1, degree + 1)
        for i in range(degree + 1):
            for k in range(degree + 1):
                hilbert[i, k] = mp.mpf(1) / (i + k + 1)
        c = mp.lu_solve(hilbert, mp.matrix(m))
        return [c[i] for i in range(degree + 1)]


@functools.lru_cache(maxsize=None)
def compute_table(degree, dps=30):
    """Fresh mpmath computation: tuple of 16 tuples of float64 coefficients (c_0..c_d)."""
    return tuple(tuple(float(c) for c in fit_interval(j, degree, dps))
                 for j in range(1, N_INTERVALS + 1))


@functools.lru_cache(maxsize=None)
def table(degree):
    """The float64 master table for degree 1 or 3: 16 rows of (c_0, ..., c_d).

    Uses the stored copy written by ``tests/golden/make_golden.py`` (which calls only
    ``compute_table``) when present, else computes it.
    """
    key = {1: "pwl16", 3: "cubic16"}[degree]
    if os.path.exists(_STORED):
        with open(_STORED) as fh:
            stored = json.load(fh)
        if key in stored:
            return tuple(tuple(float.fromhex(h) for h in row) for row in stored[key]["coefficients"])
    return compute_table(degree)


PC_BITS = 12   # 4096 cells of (0, 1); 2048 stored cell means


def compute_pconst(bits=PC_BITS, dps=40):
    """Fresh mpmath computation of the lower-half cell means (float64), cell i < 2^(bits-1)."""
    n = 2 ** (bits - 1)
    with mp.workdps(dps):
        scale = mp.mpf(2) ** bits
        dens = [mp.mpf(0)]                   # phi(Phi^{-1}(0)) = 0
        for i in range(1, n + 1):
            z = phi_inv_mp(mp.mpf(i) / scale)
            dens.append(mp.npdf(z))
        return tuple(float(scale * (dens[i] - dens[i + 1])) for i in range(n))


@functools.lru_cache(maxsize=None)
def pconst(bits=PC_BITS):
    """The float64 lower-half cell means of the piecewise-constant inverse CDF; the stored
    copy written by ``tests/golden/make_golden.py`` when present, else computed."""
    key = "pconst%d" % (2 ** bits)
    if os.path.exists(_STORED):
        with open(_STORED) as fh:
            stored = json.load(fh)
        if key in stored:
            return tuple(float.fromhex(h) for h in stored[key]["means"])
    return compute_pconst(bits)
