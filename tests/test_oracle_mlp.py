"""Pins of the oracle's MLP surrogate: gradients vs central finite differences, Adam vs its
closed form under a constant gradient, each layer of the deployed evaluation rounded once
(hand-computed one-unit networks), the bound on the second layer's two correct roundings
against sampled nearby sums, the deployed (clamp to [0, 1]) form equal to the
training (hard tanh) form in exact arithmetic, and exact mirror symmetry of the deployed
model."""

import numpy as np
import pytest

from oracle import fp, mlp


def _params(seed=0):
    # weights large enough that every unit saturates somewhere on the inputs used
    rng = np.random.default_rng(seed)
    return rng.normal(0, 1.5, mlp.N_PARAMS)


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


def test_hard_tanh_and_its_slope():
    z = np.array([-3.0, -1.0, -0.25, 0.0, 0.5, 1.0, 2.0])
    np.testing.assert_array_equal(mlp.hard_tanh(z), [-1.0, -1.0, -0.25, 0.0, 0.5, 1.0, 1.0])
    np.testing.assert_array_equal(mlp.hard_tanh_slope(z), [0, 0, 1, 1, 1, 0, 0])


def test_backprop_of_a_unit_in_its_linear_region():
    # one hidden path in the linear region: y = W3[0] (W2[0,0] (W1[0] x + b1[0]) + b2[0]) + b3
    p = np.zeros(mlp.N_PARAMS)
    W1, b1, W2, b2, W3, b3 = (0.5, 0.1, 0.8, -0.2, 1.5, 0.3)
    p[0], p[16], p[32], p[288], p[304], p[320] = W1, b1, W2, b2, W3, b3
    x = np.array([0.4])
    h1 = W1 * 0.4 + b1
    y = W3 * (W2 * h1 + b2) + b3
    got, _ = mlp.forward(p, x)
    assert got[0] == pytest.approx(y, rel=1e-15)
    _, g = mlp.loss_grad(p, x, np.array([0.0]))
    dy = 2.0 * y
    assert g[320] == pytest.approx(dy) and g[304] == pytest.approx(dy * (W2 * h1 + b2))
    assert g[32] == pytest.approx(dy * W3 * h1) and g[0] == pytest.approx(dy * W3 * W2 * 0.4)


def test_deployed_form_equals_training_form_without_rounding():
    # c = (h + 1) / 2: the folded parameters give the same y in exact arithmetic
    p = _params(4)
    q = mlp.fold(p, rounding=np.float64)
    x = np.linspace(-1.0, 1.0, 4001)
    y, _ = mlp.forward(p, x)
    A1, a1, A2, a2, A3, a3 = mlp.unpack(q)
    c1 = np.clip(np.outer(x, A1) + a1, 0.0, 1.0)
    c2 = np.clip(c1 @ A2.T + a2, 0.0, 1.0)
    np.testing.assert_allclose(c2 @ A3 + a3, y, rtol=0, atol=1e-12)
    # the binary32 fold agrees with the float64 one to binary32 rounding
    np.testing.assert_allclose(mlp.fold(p), q, rtol=1e-5, atol=1e-5)


def _one_unit_model(A1, a1, A2, a2, A3, a3):
    """Deployed parameters with only unit 0 of each layer connected."""
    z = np.zeros(16)
    W2 = np.zeros((16, 16))
    W2[0, 0] = A2
    b2 = np.zeros(16)
    b2[0] = a2
    b2[1:] = -1.0   # the other second-layer units clamp to 0
    W3 = np.zeros(16)
    W3[0] = A3
    w1, bb1 = z.copy(), z.copy()
    w1[0], bb1[0] = A1, a1
    return mlp.pack(w1, bb1, W2, b2, W3, a3)


def test_deployed_evaluation_rounds_each_layer_once():
    # x = 3/4: c1 = R16(0.5 x + 0.25) = 5/8 exactly; d = 5/8 * R16(1/3) = 5/8 * 1365 2^-12
    # = 6825 2^-15 = 1706.25 2^-13 rounds to 1706 2^-13 (spacing 2^-13 on [1/8, 1/4))
    third = float(np.float16(1.0 / 3.0))
    assert third == 1365 * 2.0 ** -12
    q = _one_unit_model(0.5, 0.25, third, 0.0, 1.0, 0.0)
    y = mlp.eval_deployed(q, np.array([0.75]))
    assert y[0] == 1706 * 2.0 ** -13
    assert abs(y[0] - 0.625 * third) == 0.25 * 2.0 ** -13      # the second layer's rounding
    # first layer: one rounding of the fused A1 x + a1 (x = 2^-11 + 2^-12: 0.5 x + 0.25 needs
    # 14 bits; R16 of it is 0.25 + 2^-12, the nearest binary16 value above 1/4 with ties even)
    q1 = _one_unit_model(0.5, 0.25, 1.0, 0.0, 1.0, 0.0)
    x = 2.0 ** -11 + 2.0 ** -12
    assert mlp.eval_deployed(q1, np.array([x]))[0] == float(np.float16(0.25 + 0.5 * x))
    # clamps: negative arguments give 0, arguments above 1 give 1
    assert mlp.eval_deployed(_one_unit_model(1.0, -0.5, 1.0, 0.0, 2.0, 0.5), np.array([0.25]))[0] == 0.5
    assert mlp.eval_deployed(_one_unit_model(1.0, 0.0, 4.0, 0.0, 2.0, 0.5), np.array([0.5]))[0] == 2.5


def test_c2_allowance_bounds_every_nearby_rounding():
    rng = np.random.default_rng(11)
    q = mlp.deployed(_params(7))
    x16 = mlp.input16(rng.uniform(0.0, 6.6, 3000))
    c1, d, A2, a2, A3, a3 = mlp._layers(q, x16)
    delta = mlp.C2_REL * (np.abs(c1) @ np.abs(A2).T + np.abs(a2))
    y = mlp.eval_deployed(q, x16)
    allow = mlp.c2_allowance(q, x16)
    assert np.all(mlp.c2_allowance(q, x16, rel=0.0) == 0.0)
    assert 0 < np.mean(allow > 0) < 0.75
    for _ in range(20):
        dd = d + delta * rng.uniform(-1.0, 1.0, d.shape)
        yy = np.clip(dd.astype(np.float16).astype(np.float64), 0.0, 1.0) @ A3 + a3
        assert np.all(np.abs(yy - y) <= allow * (1 + 1e-12))
    # a sum on a rounding boundary (d = 1706.5 2^-13 at c1 = 5/8): either neighbour, one
    # binary16 spacing apart
    third = float(np.float16(1.0 / 3.0))
    q2 = _one_unit_model(0.5, 0.25, 1.0, 0.0, 3.0, 0.0)
    A1b, a1b, A2b, a2b, A3b, a3b = mlp.unpack(q2)
    A2b[0, 0] = third
    a2b[0] = 1706.5 * 2.0 ** -13 - 0.625 * third           # exact: both multiples of 2^-15
    q2 = mlp.pack(A1b, a1b, A2b, a2b, A3b, a3b)
    assert mlp._layers(q2, np.array([0.75]))[1][0, 0] == 1706.5 * 2.0 ** -13
    assert mlp.c2_allowance(q2, np.array([0.75]))[0] == 3.0 * 2.0 ** -13


def test_deployed_model_is_mirror_symmetric_and_bounded():
    q = mlp.deployed(_params(3))
    assert np.all(q.astype(np.float16).astype(np.float64) == q)     # binary16 values
    x = np.random.default_rng(2).integers(0, 2 ** 32, 5000, dtype=np.uint64)
    z = mlp.approx_icdf(x, q, fp.FP64)
    zm = mlp.approx_icdf(np.uint64(2 ** 32 - 1) - x, q, fp.FP64)
    np.testing.assert_array_equal(zm, -z)
    A1, a1, A2, a2, A3, a3 = mlp.unpack(q)
    # |Z~| <= r + |y| with r <= sqrt(64 ln 2) for 32-bit words and c2 in [0, 1]
    assert np.abs(z).max() <= np.sqrt(64 * np.log(2.0)) + abs(a3) + np.abs(A3).sum()


def test_inference_input_and_radius():
    # 2u'' = R_32(2 xm + 1) 2^-32: word 0 gives 2^-32 exactly, the middle word rounds to 1
    r, two_u = mlp.radius(np.array([0, 2 ** 31 - 1], dtype=np.uint64))
    assert two_u[0] == 2.0 ** -32 and two_u[1] == 1.0 and r[1] == 0.0
    assert r[0] == pytest.approx(np.sqrt(64 * np.log(2.0)), rel=1e-15)
    x16 = mlp.input16(r)
    assert x16[1] == -1.0 and np.float16(x16[0]) == x16[0]
    lo, hi = mlp.input16_neighbours(np.array([0, 12345, 2 ** 31 - 1], dtype=np.uint64), 0.0)
    np.testing.assert_array_equal(lo, hi)


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


def test_payoff_allowance_bounds_perturbed_paths():
    """The first-order payoff bounds of the nested paths hold for variables moved anywhere
    within their allowances (binary32 Kahan paths, level 4, call payoff)."""
    import mlmc_workloads as W
    from oracle import mlmc, philox
    rng = np.random.default_rng(12)
    q = mlp.deployed(_params(5))
    level, n = 4, 400
    o = mlmc.level_paths(level, np.arange(n), W.GBM_CALL, rv_mode=mlmc.RV_MLP, precision=fp.FP32, nested=True,
                         kahan=True, seed=8, stream=1, mlp_params=q)
    w = philox.words(8, 1, level, 0, np.arange(n, dtype=np.uint64), 2 ** level)
    zt = mlp.approx_icdf(w, q, fp.FP32).astype(np.float64)
    allow = mlp.approx_icdf_allowance(w, q)
    assert np.mean(o["Pf_bar_allow"] > 0) > 0.2        # the bound is exercised
    cp = mlmc.constants(W.GBM_CALL, level, fp.FP32)
    for _ in range(5):
        z2 = (zt + allow * rng.uniform(-1.0, 1.0, zt.shape)).astype(np.float32)
        Xf, Xc = mlmc._paths(level, z2, lambda k: z2[:, k - 1] + z2[:, k], cp, kahan=True)
        pf = fp.to64(mlmc.payoff(Xf, mlmc.PAYOFF_CALL, cp[4]))
        pc = fp.to64(mlmc.payoff(Xc, mlmc.PAYOFF_CALL, cp[4]))
        # the perturbed paths' own rounding differs from the oracle's by a few binary32 ulps
        assert np.all(np.abs(pf - o["Pf_bar"]) <= o["Pf_bar_allow"] + 1e-6)
        assert np.all(np.abs(pc - o["Pc_bar"]) <= o["Pc_bar_allow"] + 1e-6)
