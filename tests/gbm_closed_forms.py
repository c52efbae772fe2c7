"""Closed-form level moments for geometric Brownian motion under Euler-Maruyama coupling.

Infinite-precision moments of the MLMC level differences for a(X) = mu X, b(X) = sigma X
and P(X) = X, with fine step delta = T 2^-l and coarse step 2 delta (Section 3).  One coarse
step multiplies the four coupled states by independent factors

    F_x = (a + b Z_1^x)(a + b Z_2^x),   G_x = c + b (Z_1^x + Z_2^x),
    a = 1 + mu delta,  b = sigma sqrt(delta),  c = 1 + 2 mu delta,

where x labels the exact (h) or approximate (b) variable drawn from the same uniform.  Odd
joint moments vanish by the mirror symmetry u -> 1 - u, so with k_xy = E[Z^x Z^y]:

    E[F_x F_y] = (a^2 + b^2 k_xy)^2,  E[G_x G_y] = c^2 + 2 b^2 k_xy,
    E[F_x G_y] = a^2 c + 2 a b^2 k_xy,

and second moments of products of independent steps multiply.  Used as test pins only.
"""

import math
from itertools import product


def level_moments(level, mu=0.05, sigma=0.2, x0=1.0, T=1.0, k_hh=1.0, k_hb=1.0, k_bb=1.0):
    """Means and variances of the two-way (exact and approximate) and four-way differences."""
    d = T * 2.0 ** -level
    a, b, c = 1 + mu * d, sigma * math.sqrt(d), 1 + 2 * mu * d
    kap = {("h", "h"): k_hh, ("h", "b"): k_hb, ("b", "h"): k_hb, ("b", "b"): k_bb}
    if level == 0:
        # one fine step, no coarse path: P = x0 (a + b Z)
        mean = x0 * a
        var = {"h": x0 * x0 * b * b * k_hh, "b": x0 * x0 * b * b * k_bb}
        four_var = x0 * x0 * b * b * (k_hh - 2 * k_hb + k_bb)
        return {"mean_two": mean, "var_two_exact": var["h"], "var_two_approx": var["b"],
                "mean_four": 0.0, "var_four": four_var}
    M = 2 ** (level - 1)
    states = [("f", "h"), ("c", "h"), ("f", "b"), ("c", "b")]

    def second(s1, s2):
        (p1, x1), (p2, x2) = s1, s2
        k = kap[(x1, x2)]
        if p1 == "f" and p2 == "f":
            e = (a * a + b * b * k) ** 2
        elif p1 == "c" and p2 == "c":
            e = c * c + 2 * b * b * k
        else:
            e = a * a * c + 2 * a * b * b * k
        return x0 * x0 * e ** M

    mean_f, mean_c = x0 * a ** (2 * M), x0 * c ** M
    mean_two = mean_f - mean_c
    var_two = {}
    for x in ("h", "b"):
        e2 = second(("f", x), ("f", x)) - 2 * second(("f", x), ("c", x)) + second(("c", x), ("c", x))
        var_two[x] = e2 - mean_two ** 2
    sign = {("f", "h"): 1, ("c", "h"): -1, ("f", "b"): -1, ("c", "b"): 1}
    e_four2 = sum(sign[s1] * sign[s2] * second(s1, s2) for s1, s2 in product(states, states))
    return {"mean_two": mean_two, "var_two_exact": var_two["h"], "var_two_approx": var_two["b"],
            "mean_four": 0.0, "var_four": e_four2}


def call_level0_mean(mu=0.05, sigma=0.2):
    """E[max(X_1 - 1, 0)] with X_1 = 1 + mu + sigma Z: mu Phi(mu/sigma) + sigma phi(mu/sigma)."""
    r = mu / sigma
    Phi = 0.5 * math.erfc(-r / math.sqrt(2))
    phi = math.exp(-0.5 * r * r) / math.sqrt(2 * math.pi)
    return mu * Phi + sigma * phi


def table_second_moment(tab):
    """E Z~^2 = 2 sum_j |I_j| int_0^1 q_j(t)^2 dt for a mirrored dyadic table (exact)."""
    total = 0.0
    for j, c in enumerate(tab, start=1):
        width = 2.0 ** -(j + 1) if j < 16 else 2.0 ** -16
        sq = math.fsum(ca * cb / (a + b + 1) for a, ca in enumerate(c) for b, cb in enumerate(c))
        total += width * sq
    return 2 * total


def word_law_mse(z_exact, z_approx, n_dense=2 ** 16):
    """E|Z - Z~|^2 under the law of U = (x + 1/2) 2^-32 over all 32-bit words x.

    ``z_exact`` / ``z_approx`` map uint32 word arrays to Z / Z~.  The far-tail interval
    I_16 (65536 words per side) is enumerated exactly; on I_1..I_15 the error is smooth
    and a midpoint grid of ``n_dense`` words per interval gives the word average to
    O(n_dense^-2).  The mirror doubles the lower half.
    """
    import numpy as np
    total = 0.0
    x16 = np.arange(2 ** 16, dtype=np.uint64)
    total += float(np.sum((z_exact(x16) - z_approx(x16)) ** 2)) * 2.0 ** -32
    for j in range(1, 16):
        count = 2 ** (31 - j)                        # words of I_j on the lower half
        stride = count // n_dense
        lo = 2 ** (31 - j)
        x = np.uint64(lo) + np.arange(n_dense, dtype=np.uint64) * np.uint64(stride) + np.uint64(stride // 2)
        total += float(np.mean((z_exact(x) - z_approx(x)) ** 2)) * count * 2.0 ** -32
    return 2 * total
