"""The learned approximate inverse CDF: a 1-16-16-1 tanh network (test infrastructure only).

Section 2.1 admits any approximate Gaussian variable that satisfies Assumption 2.1 (zero
mean, bounded, finite moments, bounded density with finitely many discontinuities).  This
module restates, in float64, the small network used as such an approximation:

    u' = min(u, 1 - u)                        (mirror: exact zero mean, like Figure 1)
    r  = sqrt(-2 ln(2 u'))                    (r in [0, 6.7] for 32-bit words)
    x  = r / R_SCALE - 1                      (network input)
    h1 = tanh(W1 x + b1)                      (16)
    h2 = tanh(W2 h1 + b2)                     (16 x 16)
    y  = W3 . h2 + b3                         (learns Phi^{-1}(u') + r, a smooth function
                                               of r with values in [0, 0.52])
    Z~ = y - r for u < 1/2, r - y for u >= 1/2

Z~ is bounded for the law of 32-bit words (r <= 6.7, |y| <= |b3| + sum |W3|), so
Assumption 2.1's boundedness holds.  Parameters are one flat vector of 321 values in the
order W1(16), b1(16), W2(16x16, row-major [out][in]), b2(16), W3(16), b3(1).  Training
minimises the mean squared error of y against Phi^{-1}(u') + r with Adam (Kingma and
Ba, 2015) on pairs drawn by ``training_words``.

Pinned by ``tests/test_oracle_mlp.py``: back-propagated gradients against central finite
differences, and the Adam update against its published closed form on a scalar problem.
"""

import numpy as np

from . import fp

N_HIDDEN = 16
N_PARAMS = 16 + 16 + 256 + 16 + 16 + 1
R_SCALE = 3.4
ADAM_BETA1, ADAM_BETA2, ADAM_EPS = 0.9, 0.999, 1e-8


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


def feature(u_half):
    """x = sqrt(-2 ln(2 u')) / R_SCALE - 1 for u' in (0, 1/2]."""
    u_half = np.asarray(u_half, dtype=np.float64)
    return np.sqrt(-2.0 * np.log(2.0 * u_half)) / R_SCALE - 1.0


def forward(p, x):
    """Network output y and the activations needed by ``backward``."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    x = np.asarray(x, dtype=np.float64)
    h1 = np.tanh(np.outer(x, W1) + b1)          # (B, 16)
    h2 = np.tanh(h1 @ W2.T + b2)                # (B, 16)
    y = h2 @ W3 + b3
    return y, (x, h1, h2)


def loss(p, x, target):
    """Mean squared error  (1/B) sum (y - target)^2."""
    y, _ = forward(p, x)
    return float(np.mean((y - np.asarray(target, dtype=np.float64)) ** 2))


def backward(p, cache, dy):
    """Gradient of sum_b dy_b * y_b with respect to the parameters (chain rule)."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    x, h1, h2 = cache
    dW3 = h2.T @ dy
    db3 = np.sum(dy)
    dh2 = np.outer(dy, W3)
    da2 = dh2 * (1.0 - h2 * h2)
    dW2 = da2.T @ h1
    db2 = da2.sum(axis=0)
    dh1 = da2 @ W2
    da1 = dh1 * (1.0 - h1 * h1)
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
    w = philox.words(seed, 2, 0, 0, i, 2)
    w0, w1 = w[:, 0].astype(np.uint64), w[:, 1].astype(np.uint64)
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
    """(upper-half flag, u' = min(u, 1-u)) for uint32 words, u = (x + 1/2) 2^-32."""
    x = np.asarray(x_words, dtype=np.uint64)
    s = x >= np.uint64(2 ** 31)
    xm = np.where(s, np.uint64(2 ** 32 - 1) - x, x)
    return s, (xm.astype(np.float64) + 0.5) * 2.0 ** -32


def deployed(p):
    """The inference model: parameters rounded once to binary16."""
    return np.asarray(p, dtype=np.float64).astype(np.float16).astype(np.float64)


def approx_icdf(x_words, p16, precision):
    """Z~ for uint32 words from the binary16-rounded parameters, evaluated in float64 and
    rounded once to precision p."""
    shape = np.shape(x_words)
    s, uh = mirror(np.ravel(x_words))
    r = np.sqrt(-2.0 * np.log(2.0 * uh))
    y, _ = forward(p16, r / R_SCALE - 1.0)
    q = y - r
    z = np.where(s, -q, q).reshape(shape)
    return fp.rn(precision, z)
