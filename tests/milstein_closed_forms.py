"""Closed-form level moments of geometric Brownian motion under the coupled Milstein scheme.

For dX = mu X dt + sigma X dW the Milstein step multiplies the state by

    f(Z) = a + b Z + c (Z^2 - 1),   a = 1 + mu delta,  b = sigma sqrt(delta),  c = sigma^2 delta / 2,

and the coarse step of the level coupling (Section 3: the coarse increment is the sum of two
fine ones, dW_c = sqrt(delta) S with S = Z_1 + Z_2) by

    g(S) = a_c + b S + c (S^2 - 2),   a_c = 1 + 2 mu delta.

With exact standard normal variables the second moments E[F^2], E[F G], E[G^2] of
F = f(Z_1) f(Z_2) and G = g(Z_1 + Z_2) follow from the normal moments E Z^k = (k-1)!! (k
even), computed here symbolically in exact rational arithmetic: every term with an odd
power of b has an odd normal moment and vanishes, so only b^2 = sigma^2 delta enters.
Independent steps multiply.  Used as test pins only.
"""

from fractions import Fraction

import sympy as sp


def _normal_moment(k):
    if k % 2:
        return 0
    m = 1
    for j in range(k - 1, 0, -2):
        m *= j
    return m


def _expect(expr, zs):
    """E[expr] for a polynomial in independent standard normals zs."""
    poly = sp.Poly(sp.expand(expr), *zs)
    total = sp.Integer(0)
    for powers, coeff in poly.terms():
        w = 1
        for k in powers:
            w *= _normal_moment(k)
        total += coeff * w
    return sp.simplify(total)


def step_moments(mu, sigma, delta):
    """(E F, E G, E F^2, E F G, E G^2) as exact rationals for rational mu, sigma^2, delta."""
    z1, z2, bb = sp.symbols("z1 z2 bb")  # bb stands for b, whose square is sigma^2 delta
    mu, s2, d = sp.Rational(mu), sp.Rational(sigma) ** 2, sp.Rational(delta)
    a, ac, c = 1 + mu * d, 1 + 2 * mu * d, s2 * d / 2
    f = lambda z: a + bb * z + c * (z * z - 1)  # noqa: E731
    F = f(z1) * f(z2)
    S = z1 + z2
    G = ac + bb * S + c * (S * S - 2)
    out = []
    for e in (F, G, F * F, F * G, G * G):
        v = _expect(e, [z1, z2])
        v = sp.expand(v).subs(bb ** 2, s2 * d)
        assert not v.has(bb), "odd powers of b must vanish"
        out.append(Fraction(int(sp.numer(v)), int(sp.denom(v))))
    return tuple(out)


def level_moments(level, mu="1/20", sigma="1/5", x0=1, T=1):
    """Exact mean and variance of P_l - P_{l-1} for P(X) = X (level 0: P_0 = X_1 alone)."""
    delta = Fraction(T) * Fraction(1, 2 ** level)
    mu_q, sig_q = Fraction(mu), Fraction(sigma)
    if level == 0:
        a = 1 + mu_q * delta
        b2, c = sig_q ** 2 * delta, sig_q ** 2 * delta / 2
        return {"mean": x0 * a, "var": x0 * x0 * (b2 + 2 * c * c)}
    EF, EG, EF2, EFG, EG2 = step_moments(mu_q, sig_q, delta)
    M = 2 ** (level - 1)
    mean = x0 * (EF ** M - EG ** M)
    second = x0 * x0 * (EF2 ** M - 2 * EFG ** M + EG2 ** M)
    return {"mean": mean, "var": second - mean * mean}
