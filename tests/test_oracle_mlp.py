"""Pins of the oracle's MLP surrogate: gradients vs central finite differences, Adam vs its
closed form under a constant gradient, and exact mirror symmetry of the deployed model."""

import numpy as np

from oracle import fp, mlp


def _params(seed=0):
    rng = np.random.default_rng(seed)
    return rng.normal(0, 0.5, mlp.N_PARAMS)


def test_backprop_matches_finite_differences():
    p = _params()
    rng = np.random.default_rng(1)
    uh = rng.uniform(1e-9, 0.5, 64)
    x = mlp.feature(uh)
    target = np.array([-1.0 * v for v in np.sqrt(-2 * np.log(2 * uh))])
    _, g = mlp.loss_grad(p, x, target)
    h = 1e-6
    for i in range(mlp.N_PARAMS):
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss(p + e, x, target) - mlp.loss(p - e, x, target)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), i


def test_adam_closed_form_constant_gradient():
    # with a constant gradient g the bias-corrected moments are exactly g and g^2, so
    # p_t = p_0 - t lr g / (|g| + eps)
    p0 = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -0.01, 2.0])
    m = np.zeros(3)
    v = np.zeros(3)
    p = p0.copy()
    lr = 1e-2
    for t in range(1, 6):
        p, m, v = mlp.adam_step(p, g, m, v, t, lr)
        np.testing.assert_allclose(p, p0 - t * lr * g / (np.abs(g) + mlp.ADAM_EPS), rtol=1e-12)


def test_deployed_model_is_mirror_symmetric_and_bounded():
    p16 = mlp.deployed(_params(3))
    x = np.random.default_rng(2).integers(0, 2 ** 32, 5000, dtype=np.uint64)
    z = mlp.approx_icdf(x, p16, fp.FP64)
    zm = mlp.approx_icdf(np.uint64(2 ** 32 - 1) - x, p16, fp.FP64)
    np.testing.assert_array_equal(zm, -z)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p16)
    # |Z~| <= r + |y| with r <= sqrt(64 ln 2) for 32-bit words
    assert np.abs(z).max() <= np.sqrt(64 * np.log(2.0)) + abs(b3) + np.abs(W3).sum()


def test_feature_range():
    # u' from 2^-33 (word 0) to just under 1/2
    x = mlp.feature(np.array([2.0 ** -33, 0.5 - 2.0 ** -33]))
    assert -1.0 <= x[1] < -0.99 and 0.9 < x[0] < 1.0


def test_training_pairs_cover_the_tail_and_target_the_residual():
    x, t = mlp.training_pairs(0, 0, 4096)
    xm = mlp.training_words(0, 0, 4096)
    assert np.all(xm < 2 ** 31)
    uh = (xm.astype(np.float64) + 0.5) * 2.0 ** -32
    assert np.mean(uh[1::2] < 2.0 ** -16) > 0.4          # tail-weighted odd pairs
    assert abs(np.mean(uh[0::2]) - 0.25) < 0.02           # uniform even pairs on (0, 1/2)
    assert t.min() > 0 and t.max() < 0.6                   # Phi^{-1}(u') + r in (0, 0.52]
    # the residual target is small where the leading term dominates
    assert np.all(np.abs((x + 1.0) * mlp.R_SCALE - np.sqrt(-2 * np.log(2 * uh))) < 1e-12)
