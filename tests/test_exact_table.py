"""CPU checks of the library's binary64 exact inverse CDF table (the generated header the GPU
kernels read), by the device algorithm's steps in exact rational arithmetic against mpmath:
Phi^-1(u) = x G(y), x = 2u - 1, y = 1 - x^2 rounded once, G a degree-6 polynomial in
t = y - c on y's cell (binade and five leading mantissa bits, c the cell centre).

* every cell of every binade a 32-bit word can reach has a row, and the last row is y = 1;
* at words spread over all cells (and the extreme words), the emulated result is within
  4e-16 relative of Phi^-1(u) from mpmath erfinv at 40 digits;
* the binary32-rounded leading coefficients of the cells kept in LDS are exactly binary32.
"""

import os
import re
import struct
from fractions import Fraction

import mpmath as mp
import numpy as np

HEADER = os.path.join(os.path.dirname(__file__), "..", "paper_2012_09739_amd", "csrc", "icdf_exact_coeffs.h")


def _header():
    src = open(HEADER).read()
    defs = {k: int(v) for k, v in re.findall(r"#define (MLMC_EXACT_[A-Z_]+) (\d+)", src)}
    body = src[src.index("#define MLMC_EXACT_COEFFS"):]
    vals = [float.fromhex(v) for v in re.findall(r"-?0x[0-9a-fA-F.]+p[+-]?\d+", body)]
    deg = defs["MLMC_EXACT_DEG"]
    return defs, np.array(vals).reshape(-1, deg + 1)


def _fma(a, b, c):
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def _emulate(word, defs, rows):
    cb, deg, emin = defs["MLMC_EXACT_CELL_BITS"], defs["MLMC_EXACT_DEG"], defs["MLMC_EXACT_E_MIN"]
    x = _fma(float(word), 2.0 ** -31, 2.0 ** -32 - 1.0)
    y = _fma(-x, x, 1.0)
    hi = struct.unpack("<Q", struct.pack("<d", y))[0] >> 32
    key = hi >> (20 - cb)
    c_hi = (key << (20 - cb)) | (1 << (19 - cb))
    c = struct.unpack("<d", struct.pack("<Q", c_hi << 32))[0]
    t = y - c
    assert Fraction(t) == Fraction(y) - Fraction(c)   # exact (same binade)
    co = rows[key - (emin << cb)]
    acc = co[deg]
    for j in range(deg - 1, -1, -1):
        acc = _fma(acc, t, co[j])
    return x * acc


def test_one_row_per_cell_up_to_y_equal_one():
    defs, rows = _header()
    cb, emin = defs["MLMC_EXACT_CELL_BITS"], defs["MLMC_EXACT_E_MIN"]
    assert rows.shape[0] == defs["MLMC_EXACT_ROWS"] == ((1023 - emin) << cb) + 1
    # the smallest y of a word (word 2^32 - 1: x = 1 - 2^-32, y = fma(-x, x, 1) = 2^-31 - 2^-64)
    # lies in binade E_MIN
    x = 1.0 - 2.0 ** -32
    y_min = _fma(-x, x, 1.0)
    assert y_min == 2.0 ** -31 - 2.0 ** -64
    assert 2.0 ** (emin - 1023) <= y_min < 2.0 ** (emin - 1022)
    with mp.workdps(40):
        g0 = float(mp.sqrt(mp.pi / 2))                  # G(1) = g(0), rounded once
    assert rows[-1][0] == g0 and not rows[-1][1:].any()


def test_emulated_table_against_mpmath():
    defs, rows = _header()
    rng = np.random.default_rng(11)
    words = [0, 1, 2 ** 31 - 1, 2 ** 31, 2 ** 32 - 1, 2 ** 32 - 2, 2 ** 16, 2 ** 31 + 12345]
    words += [int(w) for w in rng.integers(0, 2 ** 32, 300, dtype=np.uint64)]
    words += [int(2.0 ** e) for e in rng.uniform(0, 32, 300)]
    words += [2 ** 32 - 1 - w for w in words[:200]]
    worst = 0.0
    with mp.workdps(40):
        for w in words:
            u = (mp.mpf(w) + mp.mpf(1) / 2) / mp.mpf(2) ** 32
            ref = mp.sqrt(2) * mp.erfinv(2 * u - 1)
            got = _emulate(w, defs, rows)
            worst = max(worst, float(abs((got - ref) / ref)))
    assert worst <= 4e-16, worst


def test_lds_cells_have_binary32_leading_coefficients():
    defs, rows = _header()
    cb, emin, etop, deg = (defs["MLMC_EXACT_CELL_BITS"], defs["MLMC_EXACT_E_MIN"], defs["MLMC_EXACT_E_TOP"],
                           defs["MLMC_EXACT_DEG"])
    top = rows[(etop - emin) << cb:]
    for v in top[:, deg - 1:].ravel():
        assert float(np.float32(v)) == v
