"""Exact and approximate Gaussian variables from one uniform word (test infrastructure only).

Section 3 couples the two kinds of variable through the inverse transform method with a
shared uniform: Z_n = Phi^{-1}(U_n) and Z~_n = Phi~^{-1}(U_n) with the same U_n.

* ``exact``  : Z = Phi^{-1}(U) in float64 via SciPy's ``ndtri`` (a library primitive).
  Pinned by ``tests/test_oracle_icdf.py`` against mpmath at 40 digits, symmetry
  Phi^{-1}(1-u) = -Phi^{-1}(u), and Phi(Phi^{-1}(u)) = u.
* ``approx`` : Z~ from the dyadic piecewise polynomial of ``oracle.tables`` evaluated in
  precision p with one rounding per operation (Horner's rule, unfused).  Pinned by the
  same test file: exact mirror symmetry, boundedness, agreement with the float64
  polynomial to the rounding bound of p, interval selection by brute force against a
  direct search over the interval ends, and E Z~^2 from exact polynomial integrals against
  a direct average over a regular grid of words.

Word-to-interval map (the build's reading of the dyadic construction; u = (x + 1/2) 2^-32):
    s  = [x >= 2^31]            (upper half: mirror)
    x' = s ? 2^32 - 1 - x : x   (so u' = min(u, 1 - u) = (x' + 1/2) 2^-32 exactly)
    k  = number of leading zero bits of the 32-bit x'  (1..32)
    j  = min(k, 16)
    t  = (x' + 1/2) 2^(k+1-32) - 1   if k <= 15      (u' = 2^-(k+1) (1 + t))
         (x' + 1/2) 2^-16           otherwise        (u' = 2^-16 t)
    Z~ = s ? -q_j(t) : q_j(t)
The local coordinate is exact in float64; precision p uses R_p(t), except binary16 and
bfloat16, which use R_p(R_32(t)) (the coordinate is formed in binary32 and then narrowed).

``approx`` with RV_PCONST: the piecewise-constant variable of ``oracle.tables.pconst`` on
2^b equal cells (b = 12): with s and x' as above, cell i = x' >> (32 - b) of the lower half
(the cell of u' = (x' + 1/2) 2^-32, since the cells are aligned to the word grid) and
Z~ = s ? -m_i : m_i, m_i the cell mean rounded once to precision p.  No arithmetic.
"""

import numpy as np
from scipy.special import ndtri

from . import fp
from . import tables as _tables

RV_PWL, RV_CUBIC, RV_PCONST = 1, 2, 4
_DEGREE = {RV_PWL: 1, RV_CUBIC: 3}


def exact(x):
    """Z = Phi^{-1}((x + 1/2) 2^-32) in float64 for uint32 word(s) x."""
    u = (np.asarray(x, dtype=np.float64) + 0.5) * 2.0 ** -32
    return ndtri(u)


def clz32(v):
    """Leading zero count of 32-bit unsigned integers (32 for zero), by plain bit search."""
    v = np.asarray(v, dtype=np.uint64)
    out = np.full(v.shape, 32, dtype=np.int64)
    for b in range(31, -1, -1):
        hit = ((v >> np.uint64(b)) & np.uint64(1)).astype(bool) & (out == 32)
        out[hit] = 31 - b
    return out


def locate(x):
    """(sign_flag, interval j in 1..16, exact float64 local coordinate t) for words x."""
    x = np.asarray(x, dtype=np.uint64)
    s = x >= np.uint64(2 ** 31)
    xm = np.where(s, np.uint64(2 ** 32 - 1) - x, x)
    k = clz32(xm)
    j = np.minimum(k, 16)
    xmf = xm.astype(np.float64) + 0.5
    t = np.where(k <= 15, xmf * np.exp2((k + 1 - 32).astype(np.float64)) - 1.0, xmf * 2.0 ** -16)
    return s, j, t


def coefficients(rv_mode, precision):
    """The 16 x (d+1) coefficient table rounded once to precision p."""
    tab = np.array(_tables.table(_DEGREE[rv_mode]), dtype=np.float64)
    return fp.rn(precision, tab)


def local_coordinate(t, precision):
    if precision in (fp.FP16, fp.BF16):   # formed in binary32 and narrowed
        return fp.rn(precision, fp.rn(fp.FP32, t).astype(np.float64))
    return fp.rn(precision, t)


def pconst_cell(x, bits=_tables.PC_BITS):
    """(sign_flag, lower-half cell index) of uint32 word(s) x on 2^bits equal cells."""
    x = np.asarray(x, dtype=np.uint64)
    s = x >= np.uint64(2 ** 31)
    xm = np.where(s, np.uint64(2 ** 32 - 1) - x, x)
    return s, (xm >> np.uint64(32 - bits)).astype(np.int64)


def approx(x, rv_mode, precision):
    """Z~ = Phi~^{-1}(U) in precision p for uint32 word(s) x (Section 2.1, Lemmas 2.2/2.3)."""
    if rv_mode == RV_PCONST:
        s, i = pconst_cell(x)
        m = fp.rn(precision, np.array(_tables.pconst(), dtype=np.float64))[i]
        return fp.like(m, np.where(s, -fp.to64(m), fp.to64(m)))
    s, j, t = locate(x)
    c = coefficients(rv_mode, precision)[j - 1]          # rows of (c_0..c_d), dtype p
    tp = local_coordinate(t, precision)
    d = c.shape[-1] - 1
    q = c[..., d].copy()
    for i in range(d - 1, -1, -1):
        q = q * tp          # one rounding
        q = q + c[..., i]   # one rounding
    return fp.like(q, np.where(s, -q, q))
