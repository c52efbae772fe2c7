"""The learned approximate inverse CDF: a 1-16-16-1 piecewise-linear network (test
infrastructure only).

Section 2.1 admits any approximate Gaussian variable that satisfies Assumption 2.1 (zero
mean, bounded, finite moments, bounded density with finitely many discontinuities).  This
module restates, in float64, the small network used as such an approximation.

Training form (the binary32 master parameters), with the hard tanh ht(z) = min(max(z, -1), 1):

    u' = min(u, 1 - u)                        (mirror: exact zero mean, like Figure 1)
    r  = sqrt(-2 ln(2 u'))                    (r in [0, 6.7] for 32-bit words)
    x  = r / R_SCALE - 1                      (network input)
    h1 = ht(W1 x + b1)                        (16)
    h2 = ht(W2 h1 + b2)                       (16 x 16)
    y  = W3 . h2 + b3                         (learns Phi^{-1}(u') + r, a smooth function
                                               of r with values in [0, 0.52])
    Z~ = y - r for u < 1/2, r - y for u >= 1/2

Deployed form (what the level kernels evaluate): the same function with the clamp to [0, 1]
as activation, c = (h + 1) / 2, so that each activation is the clamp output modifier of the
instruction that forms its argument:

    c1 = clamp01(A1 x + a1),  c2 = clamp01(A2 c1 + a2),  y = A3 . c2 + a3,
    A1 = W1 / 2, a1 = (b1 + 1) / 2, A2 = W2, a2 = (b2 - W2 1 + 1) / 2, A3 = 2 W3, a3 = b3 - W3 . 1

formed in binary32 (sums in index order) and rounded once to binary16.  Inference: the input
2u' is the word's 2 xm + 1 rounded to binary32 times 2^-32, r = sqrt(-2 ln 2u'), x = r C - 1
with C = R_32(1 / R_SCALE), rounded to binary16; the first layer is one binary16 fused
multiply-add per unit (a single rounding); the 16 x 16 layer takes binary16 activations,
accumulates in binary32 (here: exactly) and its result is rounded to binary16 before the
clamp, c2 = clamp01(R_16(A2 c1 + a2)); the output layer takes those binary16 activations and
accumulates in binary32 (here: exactly).  Where A2 c1 + a2 lies so close to a rounding
boundary of binary16 that the binary32 accumulation may land on either side, both roundings
are correct; ``c2_allowance`` bounds what that can change in y.

Z~ is bounded for the law of 32-bit words (r <= 6.7, |y| <= |a3| + sum |A3|), so Assumption
2.1's boundedness holds.  Parameters are one flat vector of 321 values in the order W1(16),
b1(16), W2(16x16, row-major [out][in]), b2(16), W3(16), b3(1) (the deployed form uses the
same layout for A1, a1, A2, a2, A3, a3).  Training minimises the mean squared error of y
against Phi^{-1}(u') + r with Adam (Kingma and Ba, 2015) on pairs drawn by
``training_words``.

Pinned by ``tests/test_oracle_mlp.py``: back-propagated gradients against central finite
differences, the Adam update against its closed form on a scalar problem, and the deployed
form equal to the training form without rounding.
"""

import numpy as np

from . import fp

N_HIDDEN = 16
N_PARAMS = 16 + 16 + 256 + 16 + 16 + 1
R_SCALE = 3.4
ADAM_BETA1, ADAM_BETA2, ADAM_EPS = 0.9, 0.999, 1e-8
# the input scale of inference, 1 / R_SCALE rounded to binary32
C_INPUT = float(np.float32(1.0 / R_SCALE))


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    if p.size != N_PARAMS:
        raise ValueError("expected 321 parameters")
    o = 0
    W1 = p[o:o + 16]; o += 16
    b1 = p[o:o + 16]; o += 16
    W2 = p[o:o + 256].reshape(16, 16); o += 256
    b2 = p[o:o + 16]; o += 16
    W3 = p[o:o + 16]; o += 16
    b3 = p[o]
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([W1, b1, np.asarray(W2).reshape(-1), b2, W3, [b3]]).astype(np.float64)


def hard_tanh(z):
    return np.clip(z, -1.0, 1.0)


def hard_tanh_slope(z):
    """Derivative of the hard tanh: 1 inside (-1, 1), 0 outside (and at the kinks)."""
    return ((z > -1.0) & (z < 1.0)).astype(np.float64)


def feature(u_half):
    """x = sqrt(-2 ln(2 u')) / R_SCALE - 1 for u' in (0, 1/2] (the training input)."""
    u_half = np.asarray(u_half, dtype=np.float64)
    return np.sqrt(-2.0 * np.log(2.0 * u_half)) / R_SCALE - 1.0


def forward(p, x):
    """Network output y of the training form and the values needed by ``backward``."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    x = np.asarray(x, dtype=np.float64)
    z1 = np.outer(x, W1) + b1                   # (B, 16)
    h1 = hard_tanh(z1)
    z2 = h1 @ W2.T + b2                         # (B, 16)
    h2 = hard_tanh(z2)
    y = h2 @ W3 + b3
    return y, (x, z1, h1, z2, h2)


def loss(p, x, target):
    """Mean squared error  (1/B) sum (y - target)^2."""
    y, _ = forward(p, x)
    return float(np.mean((y - np.asarray(target, dtype=np.float64)) ** 2))


def backward(p, cache, dy):
    """Gradient of sum_b dy_b * y_b with respect to the parameters (chain rule)."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    x, z1, h1, z2, h2 = cache
    dW3 = h2.T @ dy
    db3 = np.sum(dy)
    da2 = np.outer(dy, W3) * hard_tanh_slope(z2)
    dW2 = da2.T @ h1
    db2 = da2.sum(axis=0)
    da1 = (da2 @ W2) * hard_tanh_slope(z1)
    dW1 = da1.T @ x
    db1 = da1.sum(axis=0)
    return pack(dW1, db1, dW2, db2, dW3, db3)


def loss_grad(p, x, target):
    """(MSE, its gradient) for one mini-batch."""
    y, cache = forward(p, x)
    r = y - np.asarray(target, dtype=np.float64)
    dy = 2.0 * r / r.size
    return float(np.mean(r * r)), backward(p, cache, dy)


def adam_step(p, g, m, v, step, lr):
    """One Adam update (bias-corrected first and second moments); step counts from 1."""
    m = ADAM_BETA1 * m + (1.0 - ADAM_BETA1) * g
    v = ADAM_BETA2 * v + (1.0 - ADAM_BETA2) * g * g
    mhat = m / (1.0 - ADAM_BETA1 ** step)
    vhat = v / (1.0 - ADAM_BETA2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + ADAM_EPS), m, v


def training_words(seed, first, n):
    """Mirrored words xm (u' = (xm + 1/2) 2^-32 < 1/2) of training pairs first..first+n-1.

    Pair i takes Philox words w0, w1 of counter (0, i, 2 << 16, 0) (stream 2): even pairs
    are uniform samples (w0 mirrored), odd pairs are tail-weighted: xm = (w0 >> 1) >> (w1 mod
    31), which spreads the samples over the 31 dyadic scales of (0, 1/2)."""
    from . import philox
    i = np.arange(first, first + n, dtype=np.uint64)
    seed = int(seed)
    r = philox.philox4x32_10(np.uint64(0), i, np.uint64(2 << 16), np.uint64(0), np.uint64(seed & 0xFFFFFFFF),
                             np.uint64((seed >> 32) & 0xFFFFFFFF))
    w0, w1 = r[0], r[1]
    xm_u = np.where(w0 >= np.uint64(2 ** 31), np.uint64(2 ** 32 - 1) - w0, w0)
    xm_t = (w0 >> np.uint64(1)) >> (w1 % np.uint64(31))
    return np.where(i % np.uint64(2) == 0, xm_u, xm_t)


def training_pairs(seed, first, n):
    """(x, target) of training pairs: x the network input, target Phi^{-1}(u') + r."""
    from scipy.special import ndtri
    xm = training_words(seed, first, n)
    uh = (xm.astype(np.float64) + 0.5) * 2.0 ** -32
    r = np.sqrt(-2.0 * np.log(2.0 * uh))
    return r / R_SCALE - 1.0, ndtri(uh) + r


def mirror(x_words):
    """(upper-half flag, mirrored word xm) for uint32 words: xm = 2^32 - 1 - x on the upper half."""
    x = np.asarray(x_words, dtype=np.uint64)
    s = x >= np.uint64(2 ** 31)
    return s, np.where(s, np.uint64(2 ** 32 - 1) - x, x)


def fold(p, rounding=np.float32):
    """The deployed (clamp to [0, 1]) form of training parameters p, formed in the given
    arithmetic (binary32: one rounding per operation, sums in index order; float64 for the
    unrounded algebra)."""
    f = rounding
    W1, b1, W2, b2, W3, b3 = (np.asarray(a, dtype=np.float64).astype(f) for a in unpack(p))
    b3 = f(b3)
    half, one, two = f(0.5), f(1.0), f(2.0)
    A1 = W1 * half
    a1 = (b1 + one) * half
    a2 = np.empty(16, dtype=f)
    for n in range(16):
        s = f(0.0)
        for k in range(16):
            s = f(s + W2[n, k])
        a2[n] = f(f(f(b2[n] - s) + one) * half)
    t = f(0.0)
    for k in range(16):
        t = f(t + W3[k])
    return pack(A1, a1, W2, a2, W3 * two, f(b3 - t))


def deployed(p):
    """The inference model: the deployed form of p (binary32) rounded once to binary16."""
    return fold(p).astype(np.float16).astype(np.float64)


def radius(xm):
    """(r, 2u'') with 2u'' = R_32(2 xm + 1) 2^-32 and r = sqrt(-2 ln 2u'')."""
    a = (2 * np.asarray(xm, dtype=np.uint64) + np.uint64(1)).astype(np.float32).astype(np.float64)
    two_u = a * 2.0 ** -32
    return np.sqrt(-2.0 * np.log(two_u)), two_u


def input16(r):
    """The binary16 network input R_16(r C - 1) of inference (from the unrounded r C - 1)."""
    return (r * C_INPUT - 1.0).astype(np.float16).astype(np.float64)


def _r16(v):
    """Round to binary16 (nearest, ties to even; NumPy converts float64 directly)."""
    return np.asarray(v, dtype=np.float64).astype(np.float16).astype(np.float64)


def _layers(q, x16):
    A1, a1, A2, a2, A3, a3 = unpack(q)
    c1 = np.clip(_r16(np.outer(x16, A1) + a1), 0.0, 1.0)  # one rounding of the exact A1 x + a1
    d = c1 @ A2.T + a2                                     # exact up to float64 rounding
    return c1, d, A2, a2, A3, a3


def eval_deployed(q, x16):
    """y of the deployed model q at binary16 inputs x16: the first layer's fused binary16
    multiply-add (exact in float64, rounded once), the second layer's sum exact and rounded
    once to binary16, the output layer exact."""
    c1, d, A2, a2, A3, a3 = _layers(q, np.asarray(x16, dtype=np.float64))
    return np.clip(_r16(d), 0.0, 1.0) @ A3 + a3


# binary32 accumulation of the 16 products and the bias of a second-layer unit, in any order:
# |computed - exact| <= 16 u (|a2| + sum |A2 c1|), u = 2^-24 (each of at most 16 additions
# rounds once, relative to a partial sum bounded by that total)
C2_REL = 16 * 2.0 ** -24


def c2_allowance(q, x16, rel=C2_REL):
    """Per sample, the most y can change when the binary16 rounding of a second-layer sum
    d = A2 c1 + a2 is taken from a binary32 value within delta = rel (|a2| + sum |A2 c1|) of
    d: units whose interval [d - delta, d + delta] straddles a rounding boundary of binary16
    (inside the clamp's range) may yield any clamped rounding between the two ends."""
    c1, d, A2, a2, A3, a3 = _layers(q, np.asarray(x16, dtype=np.float64))
    delta = rel * (np.abs(c1) @ np.abs(A2).T + np.abs(a2))
    lo = np.clip(_r16(d - delta), 0.0, 1.0)
    hi = np.clip(_r16(d + delta), 0.0, 1.0)
    return (hi - lo) @ np.abs(A3)


def approx_icdf(x_words, q, precision, x16=None):
    """Z~ for uint32 words from the deployed model q (binary16 values), rounded once to
    precision p.  x16 (optional) replaces the binary16 inputs of the words."""
    shape = np.shape(x_words)
    s, xm = mirror(np.ravel(x_words))
    r, _ = radius(xm)
    xi = input16(r) if x16 is None else np.ravel(x16)
    z = eval_deployed(q, xi) - r
    z = np.where(s, -z, z).reshape(shape)
    return fp.rn(precision, z)


def approx_icdf_allowance(x_words, q, x16=None, rel=C2_REL):
    """``c2_allowance`` of each word's variable (|Z~| changes as |y| does)."""
    shape = np.shape(x_words)
    _, xm = mirror(np.ravel(x_words))
    r, _ = radius(xm)
    xi = input16(r) if x16 is None else np.ravel(x16)
    return c2_allowance(q, xi, rel).reshape(shape)


def input16_neighbours(x_words, delta):
    """For each word, the binary16 roundings of every value within delta of r C - 1: (lo, hi),
    equal unless r C - 1 lies within delta of a rounding boundary of binary16."""
    _, xm = mirror(np.ravel(x_words))
    r, _ = radius(xm)
    x = r * C_INPUT - 1.0
    lo = (x - delta).astype(np.float16).astype(np.float64)
    hi = (x + delta).astype(np.float16).astype(np.float64)
    return lo, hi
