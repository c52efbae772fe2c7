"""Precision model for the oracle (test infrastructure only).

Section 2.2 assumes the standard rounding model: every floating point operation returns
the exactly rounded result under round-to-nearest-even, x (*) y = R(x * y).  The oracle
emulates binary64, binary32 and binary16 with NumPy scalars/arrays of those dtypes, one
rounding per operation:

* float64 and float32 arithmetic in NumPy is IEEE correctly rounded;
* float16 arithmetic in NumPy is computed in float32 and rounded to float16, which is the
  correctly rounded float16 result for + - x because 24 >= 2*11 + 2 (double rounding is
  innocuous when the wider format has at least 2p+2 bits; Figueroa, 1995);
* bfloat16 (8 significant bits, the exponent range of binary32; the 7-bit-mantissa format of
  the precision experiments around Figure 3) has no NumPy dtype: values are held in float64
  arrays of class ``BF16Array``, whose + - x max min round every result to 8 significant
  bits (``round_bits``), the correctly rounded result since the float64 operation on two
  8-bit operands is exact or at least 2*8+2 bits wide;
* P17, a 16-bit-mantissa format (17 significant bits; the fourth width of the same
  precision experiments, between binary16 and binary32), likewise in ``P17Array``: float64
  has 53 >= 2*17+2 bits, so rounding its result again to 17 bits is the correctly rounded
  17-bit result.  Neither emulation models subnormals or overflow (the paths stay near 1).

Nothing here uses fused multiply-add: the method's operations are the separate roundings
the paper writes.
"""

import numpy as np

FP64, FP32, FP16, BF16, P17 = 0, 1, 2, 3, 4
DTYPES = {FP64: np.float64, FP32: np.float32, FP16: np.float16}
# unit roundoff of each format (half the gap between 1 and the next representable number)
UNIT_ROUNDOFF = {FP64: 2.0 ** -53, FP32: 2.0 ** -24, FP16: 2.0 ** -11, BF16: 2.0 ** -8, P17: 2.0 ** -17}
SIGNIFICAND_BITS = {FP64: 53, FP32: 24, FP16: 11, BF16: 8, P17: 17}


def round_bits(x, p):
    """Round finite float64 value(s) to p significant bits (2 <= p <= 52), to nearest with
    ties to even, from the bit pattern: add half an ulp of the kept part (minus one unless
    the kept part is odd) and clear the dropped bits; a carry into the exponent gives the
    next binade exactly."""
    x = np.asarray(x, dtype=np.float64)
    u = x.view(np.uint64)
    d = np.uint64(53 - p)
    one = np.uint64(1)
    lsb = (u >> d) & one
    r = np.asarray((u + ((one << (d - one)) - one) + lsb) & ~((one << d) - one))
    return r.view(np.float64)


class RoundedArray(np.ndarray):
    """Values of a P-bit format held in float64: the listed ufuncs round their result to P
    significant bits (subclasses fix P)."""

    P = 53
    _ROUNDED = (np.add, np.subtract, np.multiply, np.maximum, np.minimum, np.negative, np.absolute)

    def __array_ufunc__(self, ufunc, method, *inputs, **kwargs):
        args = [a.view(np.ndarray) if isinstance(a, np.ndarray) else a for a in inputs]
        res = getattr(ufunc, method)(*args, **kwargs)
        if method == "__call__" and ufunc in self._ROUNDED:
            return round_bits(res, self.P).view(type(self))
        return res


class BF16Array(RoundedArray):
    """bfloat16 values held in float64 (8 significant bits)."""
    P = 8


class P17Array(RoundedArray):
    """16-bit-mantissa values held in float64 (17 significant bits)."""
    P = 17


_EMULATED = {BF16: BF16Array, P17: P17Array}


def bf16(x):
    """R_bf16(x) of float64 value(s) as a BF16Array (one correctly rounded conversion)."""
    return round_bits(x, 8).view(BF16Array)


def p17(x):
    """R_17(x) of float64 value(s) as a P17Array (one correctly rounded conversion)."""
    return round_bits(x, 17).view(P17Array)


def dtype(precision):
    """The constructor of values of precision p (a NumPy scalar type, or an emulated format)."""
    if precision in _EMULATED:
        return bf16 if precision == BF16 else p17
    return DTYPES[precision]


def rn(precision, x):
    """R_p(x): round float64 value(s) x to precision p (one correctly rounded conversion)."""
    if precision in _EMULATED:
        return dtype(precision)(x)
    return np.asarray(x, dtype=np.float64).astype(DTYPES[precision])


def full(value, n):
    """n copies of a value of some precision, in that precision."""
    if isinstance(value, RoundedArray):
        return np.full(n, float(value)).view(type(value))
    return np.full(n, value, dtype=np.asarray(value).dtype)


def like(ref, values):
    """values (exactly representable in ref's precision) converted to ref's precision."""
    if isinstance(ref, RoundedArray):
        return np.asarray(values, dtype=np.float64).view(type(ref))
    return np.asarray(values).astype(np.asarray(ref).dtype)


def to64(x):
    """Exact conversion to plain float64 (differences are formed in binary64)."""
    return np.array(np.asarray(x, dtype=np.float64), dtype=np.float64, copy=True).view(np.ndarray)
