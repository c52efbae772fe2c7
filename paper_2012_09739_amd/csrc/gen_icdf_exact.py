"""Generates icdf_exact_coeffs.h: coefficients of the binary64 inverse normal CDF.

The device routine computes Phi^{-1}(u) = x g(w) with x = 2u - 1, y = (1-x)(1+x) rounded
once and w = -log y, where g(w) = sqrt(2) erfinv(x) / x is an entire function of w
(x^2 = 1 - e^{-w}).  It never forms w: the composition G(y) = g(-log y) is tabulated
directly on cells of y.  A cell is a binade [2^(E-1023), 2^(E-1022)) of y (E its biased
exponent) split into 2^CELL_BITS equal parts by the leading mantissa bits, so the 11
exponent bits and the CELL_BITS leading mantissa bits of y's upper word index the table
and the cell centre c is y's upper word with the bits below them replaced by one half.
On each cell G is a polynomial of degree DEG in t = y - c (exact: y and c share the
binade).  Its only singularity, y = 0, lies 2^(CELL_BITS+1) to 2^(CELL_BITS+2) half-widths
from the centre, which bounds the degree needed.  The binades run from the one holding the
smallest y of a 32-bit word, y = 1 - (1 - 2^-32)^2 (E = 991), to [1/2, 1); one more row,
the first cell of the binade [1, 2), holds the constant G(1) = g(0) for the y = 1 that
|x| < 2^-27 rounds to.

Coefficients are Chebyshev interpolants computed in 50-digit mpmath and rounded once to
binary64; on the cells of y >= 2^-10 (E >= E_TOP, the ones kept in LDS) the two leading
coefficients are rounded once more, to binary32: their terms are below 2^-30 of G there, so
binary32 costs nothing and a cell's coefficients fit 48 bytes.  The script evaluates every
cell's binary64 Horner form (correctly rounded fmas) with the stored coefficients against
mpmath and refuses to write a table whose maximum relative error exceeds 3e-16.

The log1p polynomial of the table-driven -log used by the learned variable's input
(y = 2^e m, m in [1/2, 1) split into 256 cells with centres c_i, r = m F_i - 1 for
F_i = R(1/c_i), log m = -log F_i + log1p(r), |r| <= 2^-9) is fitted here too.

Run from the repository root: python paper_2012_09739_amd/csrc/gen_icdf_exact.py
"""

import os
from fractions import Fraction

import mpmath as mp
import numpy as np

mp.mp.dps = 50
CELL_BITS = 5       # 32 cells per binade of y
DEG = 6
E_MIN = 991         # biased exponent of y = 2^-31 - 2^-64 (the word 2^32 - 1)
E_ONE = 1023        # y = 1
E_TOP = 1013        # y >= 2^-10: binary32 leading coefficients
CHECK_POINTS = 48   # evaluation points per cell, both ends included


def g_of_w(w):
    w = mp.mpf(w)
    if w == 0:
        return mp.sqrt(mp.pi / 2)
    x = mp.sqrt(-mp.expm1(-w))
    return mp.sqrt(2) * mp.erfinv(x) / x


def fma(a, b, c):
    """Correctly rounded a b + c in binary64."""
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def horner(coeffs, t):
    acc = coeffs[-1]
    for c in reversed(coeffs[:-1]):
        acc = fma(acc, t, c)
    return acc


def cheb_monomial(fn, a, b, n):
    """Chebyshev interpolant of fn on [a, b] (a < 0 < b), as monomials in t, solved in the
    scaled variable t / h for conditioning."""
    a, b = mp.mpf(a), mp.mpf(b)
    mid, h = (a + b) / 2, (b - a) / 2
    nodes = [mid + h * mp.cos(mp.pi * (k + mp.mpf(1) / 2) / (n + 1)) for k in range(n + 1)]
    V = mp.matrix(n + 1, n + 1)
    for i, t in enumerate(nodes):
        for j in range(n + 1):
            V[i, j] = (t / h) ** j
    c = mp.lu_solve(V, mp.matrix([fn(t) for t in nodes]))
    return [float(c[j] / h ** j) for j in range(n + 1)]


def cell_rows():
    """Coefficients of every cell (binade-major, then cell), the row of y = 1 last, and the
    worst relative error of their binary64 evaluation."""
    rows, worst = [], 0.0
    n_cells = 2 ** CELL_BITS
    for E in range(E_MIN, E_ONE):
        base = mp.mpf(2) ** (E - 1023)
        for j in range(n_cells):
            a = base * (1 + mp.mpf(j) / n_cells)
            b = base * (1 + mp.mpf(j + 1) / n_cells)
            c = base * (1 + (mp.mpf(j) + mp.mpf(1) / 2) / n_cells)
            cf = float(c)
            assert mp.mpf(cf) == c
            coeffs = cheb_monomial(lambda t, c=c: g_of_w(-mp.log(c + t)), a - c, b - c, DEG)
            if E >= E_TOP:
                coeffs[DEG - 1:] = [float(np.float32(v)) for v in coeffs[DEG - 1:]]
            for q in range(CHECK_POINTS + 1):
                y = float(a + (b - a) * q / CHECK_POINTS)
                if y >= float(b):
                    y = float(mp.mpf(b) * (1 - mp.mpf(2) ** -53))
                ref = g_of_w(-mp.log(mp.mpf(y)))
                worst = max(worst, float(abs((horner(coeffs, y - cf) - ref) / ref)))
            rows.append(coeffs)
    rows.append([float(g_of_w(0))] + [0.0] * DEG)
    return rows, worst


# table-driven log (Tang): the frexp mantissa m in [1/2, 1) split in 256 cells, r = m F_i - 1
# with |r| <= 2^-9, log(1 + r) = r + r^2 P(r), P fitted on [-RMAX, RMAX]
RMAX = 2.0 ** -9 * 1.001
DEG_LOG1P = 3


def p_of_r(r):
    r = mp.mpf(r)
    if abs(r) < mp.mpf(10) ** -20:  # series: the quotient below would cancel every digit
        return -mp.mpf(1) / 2 + r / 3 - r * r / 4
    return (mp.log1p(r) - r) / (r * r)


def check_log1p(coeffs, npts=4000):
    worst = 0.0
    for k in range(npts + 1):
        r = -RMAX + 2 * RMAX * k / npts
        acc = coeffs[-1]
        for c in reversed(coeffs[:-1]):
            acc = acc * r + c
        approx = (r * r) * acc + r
        worst = max(worst, float(abs(mp.mpf(approx) - mp.log1p(mp.mpf(r)))))
    return worst


def log1p_coeffs():
    a, b = -mp.mpf(RMAX), mp.mpf(RMAX)
    nodes = [b * mp.cos(mp.pi * (k + mp.mpf(1) / 2) / (DEG_LOG1P + 1)) for k in range(DEG_LOG1P + 1)]
    V = mp.matrix(DEG_LOG1P + 1, DEG_LOG1P + 1)
    for i, t in enumerate(nodes):
        for j in range(DEG_LOG1P + 1):
            V[i, j] = t ** j
    c = mp.lu_solve(V, mp.matrix([p_of_r(t) for t in nodes]))
    assert a == -b
    return [float(c[i]) for i in range(DEG_LOG1P + 1)]


def main():
    pc = log1p_coeffs()
    el1p = check_log1p(pc)
    if el1p > 2e-18:
        raise SystemExit("log1p fit not accurate enough: %g" % el1p)
    rows, worst = cell_rows()
    if worst > 3e-16:
        raise SystemExit("cell fit not accurate enough: %g" % worst)
    here = os.path.dirname(os.path.abspath(__file__))
    with open(os.path.join(here, "icdf_exact_coeffs.h"), "w") as fh:
        fh.write("// Generated by gen_icdf_exact.py (mpmath Chebyshev fits); do not edit.\n")
        fh.write("// Phi^-1(u) = x G(y), x = 2u - 1, y = (1-x)(1+x), G(y) = g(-log y) piecewise in y.\n")
        fh.write("#pragma once\n\n")
        fh.write("// log1p on |r| <= 2^-9: max absolute error %.2e\n" % el1p)
        fh.write("#define MLMC_LOG1P_DEG %d\n" % DEG_LOG1P)
        fh.write("#define MLMC_LOG1P_COEFFS { \\\n")
        for i, c in enumerate(pc):
            fh.write("    %s%s \\\n" % (float(c).hex(), "," if i + 1 < len(pc) else ""))
        fh.write("}\n")
        fh.write("// G on the cells of y: 2^CELL_BITS cells per binade, biased exponents E_MIN..1022, then\n")
        fh.write("// the row of y = 1; a degree-DEG polynomial in t = y - c per cell.  Max relative\n")
        fh.write("// error of the binary64 Horner evaluation %.2e\n" % worst)
        fh.write("#define MLMC_EXACT_CELL_BITS %d\n" % CELL_BITS)
        fh.write("#define MLMC_EXACT_DEG %d\n" % DEG)
        fh.write("#define MLMC_EXACT_E_MIN %d\n" % E_MIN)
        fh.write("// cells of biased exponent >= E_TOP: coefficients DEG-1 and DEG are binary32 values\n")
        fh.write("#define MLMC_EXACT_E_TOP %d\n" % E_TOP)
        fh.write("#define MLMC_EXACT_ROWS %d\n" % len(rows))
        fh.write("// row-major: entry k * (DEG + 1) + j is coefficient j of row k\n")
        fh.write("#define MLMC_EXACT_COEFFS { \\\n")
        flat = [v for r in rows for v in r]
        for i in range(0, len(flat), 4):
            row = ", ".join(float(v).hex() for v in flat[i:i + 4])
            fh.write("    %s%s \\\n" % (row, "," if i + 4 < len(flat) else ""))
        fh.write("}\n")
    print("rows %d x degree %d: worst %.3e; log1p %.3e" % (len(rows), DEG, worst, el1p))


if __name__ == "__main__":
    main()
