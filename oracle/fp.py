"""Precision model for the oracle (test infrastructure only).

Section 2.2 assumes the standard rounding model: every floating point operation returns
the exactly rounded result under round-to-nearest-even, x (*) y = R(x * y).  The oracle
emulates binary64, binary32 and binary16 with NumPy scalars/arrays of those dtypes, one
rounding per operation:

* float64 and float32 arithmetic in NumPy is IEEE correctly rounded;
* float16 arithmetic in NumPy is computed in float32 and rounded to float16, which is the
  correctly rounded float16 result for + - x because 24 >= 2*11 + 2 (double rounding is
  innocuous when the wider format has at least 2p+2 bits; Figueroa, 1995).

Nothing here uses fused multiply-add: the method's operations are the separate roundings
the paper writes.
"""

import numpy as np

FP64, FP32, FP16 = 0, 1, 2
DTYPES = {FP64: np.float64, FP32: np.float32, FP16: np.float16}
# unit roundoff of each format (half the gap between 1 and the next representable number)
UNIT_ROUNDOFF = {FP64: 2.0 ** -53, FP32: 2.0 ** -24, FP16: 2.0 ** -11}


def dtype(precision):
    return DTYPES[precision]


def rn(precision, x):
    """R_p(x): round float64 value(s) x to precision p (one correctly rounded conversion)."""
    return np.asarray(x, dtype=np.float64).astype(DTYPES[precision])
