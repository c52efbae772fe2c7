"""Coupled fine/coarse Euler-Maruyama paths and MLMC level corrections (test infrastructure only).

Restates, one rounding per operation, what the GPU library computes for one MLMC level:

* Euler-Maruyama in finite precision (Section 2.2): X <- X (+) (A (+) B) with
  A = a(X) (x) delta and B = (b(X) (x) sqrt(delta)) (x) Z.  For geometric Brownian motion
  a(X) = mu X, b(X) = sigma X (the test problem of Section 2.2, mu = 0.05, sigma = 0.2,
  X_0 = 1).  Reading: the constants are folded, A = ca (x) X and B = (cb (x) X) (x) Z with
  ca = R_p(mu delta) and cb = R_p(sigma sqrt(delta)) formed in binary64 and rounded once.
* Kahan-compensated state update (Section 2.3, Algorithm 1 and Code 1): with increment dX
  and compensation c,  y = dX (-) c;  s = X (+) y;  c = (s (-) X) (-) y;  X = s.
  Every low-precision path (fine and coarse) carries its own compensation; binary64
  paths never use it.
* Level coupling (Section 3): fine step delta_f = T 2^-l, coarse step 2 delta_f; the
  coarse Wiener increment is the pairwise sum of the two fine ones, so with the fine
  cb the coarse update uses Zc = Z_{2m} (+) Z_{2m+1} and ca_c = R_p(mu 2 delta_f); exact
  and approximate paths use the same uniforms; level 0 has no coarse path (P_{-1} = 0).
* Differences (Section 3): the two-way P_l - P_{l-1} and the nested four-way
  (P^_l - P^_{l-1}) - (P-_l - P-_{l-1}); the exact pair is binary64 with exact variables,
  the approximate pair runs in precision p with approximate variables.  Differences are
  formed in binary64 from the payoffs (a low-precision payoff converts exactly).
* Milstein variant (named in Section 2 among the usual schemes; Section 4 discusses its
  order-1 strong convergence, which moves the MLMC work to the coarse levels).  For GBM,
  b b' = sigma^2 X, and the scheme adds (1/2) sigma^2 X (dW^2 - delta) to the
  Euler-Maruyama increment.  Reading (the paper gives no finite-precision form):
  M = (cm (x) X) (x) (Z (x) Z (-) k) with cm = R_p(sigma^2 delta_f / 2) and
  dX = (A (+) B) (+) M; on the fine path k = 1, on the coarse path Zc = Z_{2m} (+) Z_{2m+1}
  is the coarse increment over sqrt(delta_f), so dW_c^2 - 2 delta_f = delta_f (Zc^2 - 2) and
  the same cm serves with k = 2.  k is exact in every format.
* Optional rounding diagnostic (Lemma 2.6): X-_N (precision p, approximate variables)
  minus X~_N (binary64 arithmetic with the same approximate variables evaluated in
  binary64), isolating the rounding error of the low-precision path.

Pinned by ``tests/test_oracle_mlmc.py``: GBM closed forms for the level means and
variances (exact moment recursions), the telescoping sum, the four-way identity, Kahan
exact cases, and a scalar pure-Python re-derivation on tiny inputs.
"""

import math

import numpy as np

from . import fp, icdf, philox
from . import mlp as _mlp

RV_EXACT, RV_PWL, RV_CUBIC, RV_MLP, RV_PCONST = 0, 1, 2, 3, 4
SCHEME_EM, SCHEME_MILSTEIN = 0, 1
PAYOFF_X, PAYOFF_CALL = 0, 1
TERM_TWO_WAY, TERM_FOUR_WAY, TERM_TWO_WAY_EXACT, TERM_ROUNDING = 0, 1, 2, 3


def constants(sde, level, precision):
    """(ca_f, ca_c, cb, x0, K, cm) rounded once to precision p from binary64 values."""
    dt_f = float(sde["T"]) * 2.0 ** -level
    ca_f = sde["mu"] * dt_f
    ca_c = sde["mu"] * (2.0 * dt_f)
    cb = sde["sigma"] * math.sqrt(dt_f)
    cm = 0.5 * sde["sigma"] * sde["sigma"] * dt_f
    d = fp.dtype(precision)
    return (d(ca_f), d(ca_c), d(cb), d(sde["x0"]), d(sde.get("strike", 1.0)), d(cm))


def kahan_add(a, x, c):
    """One step of Kahan compensated summation (Algorithm 1): returns (a_new, c_new)."""
    y = x - c
    a_new = a + y
    c = (a_new - a) - y
    return a_new, c


def kahan_sum(xs, dtype):
    """Algorithm 1 over a sequence, every operation rounded to ``dtype``."""
    a = dtype(0)
    c = dtype(0)
    for x in xs:
        a, c = kahan_add(a, dtype(x), c)
    return a


def em_update(X, Z, ca, cb, comp=None):
    """One Euler-Maruyama state update in the dtype of X (one rounding per operation);
    with a compensation array the update X <- X + dX is Kahan-compensated (Code 1)."""
    A = ca * X
    B = (cb * X) * Z
    dX = A + B
    if comp is None:
        return X + dX, None
    return kahan_add(X, dX, comp)


def milstein_update(X, Z, ca, cb, cm, k, comp=None):
    """One Milstein state update for GBM in the dtype of X: dX = (A (+) B) (+) M with
    M = (cm (x) X) (x) (Z (x) Z (-) k); k = 1 on the fine path, 2 on the coarse path."""
    A = ca * X
    B = (cb * X) * Z
    M = (cm * X) * (Z * Z - k)
    dX = (A + B) + M
    if comp is None:
        return X + dX, None
    return kahan_add(X, dX, comp)


def payoff(X, kind, K):
    """P(X) in the dtype of X: X itself, or the call max(X (-) K, 0)."""
    if kind == PAYOFF_X:
        return X
    return np.maximum(X - K, np.zeros_like(X))


def _paths(level, Z, Zc_sum, consts, kahan, scheme=SCHEME_EM):
    """Fine and coarse terminal states of one path pair; Z has shape (paths, steps)."""
    ca_f, ca_c, cb, x0, _, cm = consts
    n_paths, n_steps = Z.shape
    Xf = fp.full(x0, n_paths)
    Xc = fp.full(x0, n_paths)
    cf = fp.full(x0 - x0, n_paths) if kahan else None
    cc = fp.full(x0 - x0, n_paths) if kahan else None
    if scheme == SCHEME_MILSTEIN:
        one, two = fp.like(x0, 1.0), fp.like(x0, 2.0)    # exact in every format
        fine = lambda X, z, c: milstein_update(X, z, ca_f, cb, cm, one, c)  # noqa: E731
        coarse = lambda X, z, c: milstein_update(X, z, ca_c, cb, cm, two, c)  # noqa: E731
    else:
        fine = lambda X, z, c: em_update(X, z, ca_f, cb, c)  # noqa: E731
        coarse = lambda X, z, c: em_update(X, z, ca_c, cb, c)  # noqa: E731
    for n in range(n_steps):
        Xf, cf = fine(Xf, Z[:, n], cf)
        if level >= 1 and n % 2 == 1:
            Xc, cc = coarse(Xc, Zc_sum(n), cc)
    return Xf, Xc


def _mlp_payoff_allowance(level, Zt, allow, consts, Xf, Xc):
    """Bounds on |P(X_N)| changes of the fine and the coarse path when each learned variable
    Z~_n may move by allow_n (the two correct binary16 roundings of a second-layer sum).

    Euler-Maruyama for GBM multiplies the state by f_n = 1 + ca + cb Z~_n per step, so to first
    order dX_N / dZ~_n = cb X_N / f_n (coarse: the pair sum enters once, with the coarse
    factor); the payoffs are 1-Lipschitz.  A factor 1.5 covers the second-order terms and the
    rounding of the perturbed path (allow_n cb is below 1e-3 here)."""
    ca_f, ca_c, cb = (float(consts[0]), float(consts[1]), float(consts[2]))
    Zt = fp.to64(Zt)
    ff = 1.0 + ca_f + cb * Zt
    fine = cb * np.abs(Xf) * np.sum(allow / np.abs(ff), axis=1)
    if level == 0:
        return 1.5 * fine, np.zeros_like(fine)
    Zc = Zt[:, 0::2] + Zt[:, 1::2]
    fc = np.repeat(1.0 + ca_c + cb * Zc, 2, axis=1)
    coarse = cb * np.abs(Xc) * np.sum(allow / np.abs(fc), axis=1)
    return 1.5 * fine, 1.5 * coarse


def level_paths(level, paths, sde, *, rv_mode, precision, nested, kahan, seed,
                stream=0, pset=0, diag=False, mlp_params=None, scheme=SCHEME_EM):
    """Per-path payoffs and terms of one MLMC level for the given path indices.

    Returns a dict of float64 arrays: ``Pf_hat``, ``Pc_hat`` (exact pair, when computed),
    ``Pf_bar``, ``Pc_bar`` (approximate pair, when computed), ``Xf_bar``, ``Xf_tilde``
    (diagnostic) and ``terms`` of shape (4, paths) (NaN where a term is not computed).
    """
    if rv_mode == RV_EXACT and (precision != fp.FP64 or nested):
        raise ValueError("the exact (plain) estimator runs in binary64 and is not nested")
    paths = np.asarray(paths, dtype=np.uint64)
    n_steps = 2 ** level
    w = philox.words(seed, stream, level, pset, paths, n_steps)
    out = {}
    terms = np.full((4, paths.size), np.nan)
    kind = sde.get("payoff", PAYOFF_X)

    def coarse_of(Zarr):
        return lambda n: Zarr[:, n - 1] + Zarr[:, n]

    if rv_mode == RV_EXACT or nested:
        c64 = constants(sde, level, fp.FP64)
        Z = icdf.exact(w)
        Xf, Xc = _paths(level, Z, coarse_of(Z), c64, kahan=False, scheme=scheme)
        Pf = payoff(Xf, kind, c64[4])
        Pc = payoff(Xc, kind, c64[4]) if level >= 1 else np.zeros_like(Pf)
        out["Pf_hat"], out["Pc_hat"] = Pf, Pc
        two_hat = Pf - Pc
        if rv_mode == RV_EXACT:
            terms[TERM_TWO_WAY] = two_hat
        else:
            terms[TERM_TWO_WAY_EXACT] = two_hat

    if rv_mode != RV_EXACT:
        cp = constants(sde, level, precision)
        if rv_mode == RV_MLP:
            Zt = _mlp.approx_icdf(w, mlp_params, precision)
        else:
            Zt = icdf.approx(w, rv_mode, precision)
        Xf, Xc = _paths(level, Zt, coarse_of(Zt), cp, kahan=kahan and precision != fp.FP64,
                        scheme=scheme)
        Pf = fp.to64(payoff(Xf, kind, cp[4]))
        Pc = fp.to64(payoff(Xc, kind, cp[4])) if level >= 1 else np.zeros(paths.size)
        out["Pf_bar"], out["Pc_bar"] = Pf, Pc
        if rv_mode == RV_MLP and scheme == SCHEME_EM:
            out["Pf_bar_allow"], out["Pc_bar_allow"] = _mlp_payoff_allowance(
                level, Zt, _mlp.approx_icdf_allowance(w, mlp_params), cp, fp.to64(Xf), fp.to64(Xc))
        out["Xf_bar"] = fp.to64(Xf)
        two_bar = Pf - Pc
        terms[TERM_TWO_WAY] = two_bar
        if nested:
            terms[TERM_FOUR_WAY] = terms[TERM_TWO_WAY_EXACT] - two_bar
        if diag:
            c64 = constants(sde, level, fp.FP64)
            if rv_mode == RV_MLP:
                Zt64 = _mlp.approx_icdf(w, mlp_params, fp.FP64)
            else:
                Zt64 = icdf.approx(w, rv_mode, fp.FP64)
            Xt, _ = _paths(level, Zt64, coarse_of(Zt64), c64, kahan=False, scheme=scheme)
            out["Xf_tilde"] = Xt
            terms[TERM_ROUNDING] = out["Xf_bar"] - Xt
    out["terms"] = terms
    return out


def level_sums(level, n_paths, sde, *, path_offset=0, **kw):
    """Sums and sums of squares of each term over paths path_offset .. +n_paths-1.

    The sums are exactly rounded (``math.fsum``).  Returns dict(sum=[4], sumsq=[4],
    n_paths, path_steps) with NaN for terms the mode does not compute.
    """
    paths = np.arange(path_offset, path_offset + n_paths, dtype=np.uint64)
    r = level_paths(level, paths, sde, **kw)
    s, q = [], []
    for t in r["terms"]:
        if np.all(np.isnan(t)):
            s.append(math.nan)
            q.append(math.nan)
        else:
            s.append(math.fsum(t.tolist()))
            q.append(math.fsum((t * t).tolist()))
    return {"sum": s, "sumsq": q, "n_paths": n_paths, "path_steps": n_paths * 2 ** level}


def mean_var(total, total_sq, m):
    """Sample mean and unbiased sample variance from a sum and a sum of squares."""
    mean = total / m
    var = (total_sq - total * total / m) / (m - 1) if m > 1 else math.nan
    return mean, var
