"""GPU tests of the learned approximate inverse CDF: training pairs, gradients and the Adam
step against the float64 oracle, inference parity on seeded weights, and what the trained
network gains over the piecewise-linear table (approximation error, four-way variance and
the equal-variance time of the nested estimator)."""

import numpy as np
import pytest
import torch  # noqa: F401

import mlmc_workloads as W
from gpu_util import gpu_icdf, gpu_paths, torch_cuda
from oracle import fp, icdf, mlmc, mlp
from test_gpu_parity import close

import paper_2012_09739_amd as M
from paper_2012_09739_amd import estimators as E

pytestmark = pytest.mark.gpu


def dev(a, dtype=None):
    torch = torch_cuda()
    return torch.tensor(np.asarray(a), dtype=dtype or torch.float32, device="cuda")


def test_training_pairs_match_oracle():
    torch = torch_cuda()
    n, first = 5000, 123
    words = torch.zeros(n, dtype=torch.int32, device="cuda")
    x = torch.zeros(n, dtype=torch.float32, device="cuda")
    t = torch.zeros(n, dtype=torch.float32, device="cuda")
    M.mlmc_mlp_pairs(7, first, n, x, t, d_words=words)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(words.cpu().numpy().view(np.uint32), mlp.training_words(7, first, n))
    xo, to = mlp.training_pairs(7, first, n)
    np.testing.assert_allclose(x.cpu().numpy(), xo, atol=2e-7, rtol=0)
    np.testing.assert_allclose(t.cpu().numpy(), to, atol=1e-7, rtol=1e-6)


def test_gradient_matches_oracle_and_finite_differences():
    torch = torch_cuda()
    p = W.mlp_initial_params(3) + np.random.default_rng(4).normal(0, 0.05, mlp.N_PARAMS)
    n = 4096
    grad = torch.zeros(mlp.N_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    M.mlmc_mlp_grad(dev(p), 0, 0, n, grad, loss)
    g = grad.cpu().numpy().astype(np.float64)
    # the oracle differentiates the binary32-rounded parameters the GPU received
    p32 = p.astype(np.float32).astype(np.float64)
    xo, to = mlp.training_pairs(0, 0, n)
    lo, go = mlp.loss_grad(p32, xo, to)
    assert abs(float(loss.cpu()) - lo) <= 1e-4 * lo + 1e-9
    assert np.max(np.abs(g - go)) <= 1e-3 * np.max(np.abs(go))
    # and the analytic oracle gradient agrees with central differences on a few entries
    for i in (0, 20, 100, 300, 320):
        e = np.zeros_like(p32)
        e[i] = 1e-6
        fd = (mlp.loss(p32 + e, xo, to) - mlp.loss(p32 - e, xo, to)) / 2e-6
        assert abs(fd - go[i]) <= 1e-5 * max(1.0, abs(fd))


def test_first_adam_step_matches_oracle():
    torch = torch_cuda()
    p = W.mlp_initial_params(1)
    params = dev(p)
    cfg = M.mlp_cfg(seed=0, n_pairs=4096, batch=4096, epochs=1, lr=1e-3, lr_final=1e-3)
    M.mlmc_mlp_train(cfg, params)
    got = params.cpu().numpy().astype(np.float64)
    p32 = p.astype(np.float32).astype(np.float64)
    xo, to = mlp.training_pairs(0, 0, 4096)
    _, go = mlp.loss_grad(p32, xo, to)
    want, _, _ = mlp.adam_step(p32, go, np.zeros_like(go), np.zeros_like(go), 1, 1e-3)
    big = np.abs(go) > 1e-4       # the first step is -lr sign(g) where |g| >> eps
    np.testing.assert_allclose(got[big], want[big], atol=2e-6, rtol=0)
    assert np.all(np.abs(got - p32) <= 1e-3 * 1.001)


# bound on |x_gpu - x| for the network input before its binary16 rounding: r from the
# hardware base-2 logarithm and square root within a few binary32 ulps (r <= 6.7), times
# C = 0.294, plus the binary32 rounding of r C - 1
FEATURE_DELTA = 1e-6


def test_inference_matches_oracle_on_seeded_weights():
    """The learned variable against the oracle's deployed model.  Two roundings are taken
    from values the hardware may form in either of two correct ways: where the network input
    r C - 1 lies within FEATURE_DELTA of a binary16 rounding boundary, either rounding of it is
    a correct binary16 input, and where a second-layer sum lies that close to one (within the
    bound of any binary32 accumulation order), either rounding of it is; the variable must
    match the oracle for one of the two inputs, within the tolerance plus the oracle's bound
    on what the second-layer roundings can change."""
    torch = torch_cuda()
    p = W.mlp_initial_params(5) + np.random.default_rng(6).normal(0, 0.1, mlp.N_PARAMS)
    M.mlmc_mlp_load(dev(p))
    rng = np.random.default_rng(9)
    words = np.concatenate([rng.integers(0, 2 ** 32, 20000, dtype=np.uint64),
                            np.array([0, 1, 2 ** 31 - 1, 2 ** 31, 2 ** 32 - 1], dtype=np.uint64)])
    q = mlp.deployed(p.astype(np.float32))
    lo, hi = mlp.input16_neighbours(words, FEATURE_DELTA)
    assert np.mean(lo != hi) < 0.01
    want = [mlp.approx_icdf(words, q, fp.FP64, x16=x16) for x16 in (lo, hi)]
    allow = [mlp.approx_icdf_allowance(words, q, x16=x16) for x16 in (lo, hi)]
    # the second-layer rounding is decided exactly for most words
    assert np.mean(allow[0] > 0) < 0.75 and np.max(allow[0]) < 2e-3
    for prec in (M.MLMC_FP64, M.MLMC_FP32, M.MLMC_FP16):
        got = gpu_icdf(words, M.MLMC_RV_MLP, prec)
        tol = 1e-5 if prec != M.MLMC_FP16 else 4e-3
        ok = (np.abs(got - want[0]) <= tol + allow[0]) | (np.abs(got - want[1]) <= tol + allow[1])
        assert np.all(ok), (prec, words[~ok][:5], got[~ok][:5], want[0][~ok][:5])
        if prec == M.MLMC_FP32:
            exact = (allow[0] == 0) & (lo == hi)
            assert np.all(np.abs(got[exact] - want[0][exact]) <= tol)
    zm = gpu_icdf(np.uint64(2 ** 32 - 1) - words, M.MLMC_RV_MLP, M.MLMC_FP32)
    np.testing.assert_array_equal(zm, -gpu_icdf(words, M.MLMC_RV_MLP, M.MLMC_FP32))


@pytest.mark.parametrize("level", [0, 1, 4])
def test_nested_mlp_paths_match_oracle(level):
    """Per-path payoffs of the nested estimator with the learned variable: the exact pair to
    1e-13, the approximate pair to the binary32 bar plus the oracle's first-order bound on
    what the two correct roundings of each variable's second-layer sums can change (levels 0
    and 1: the shared-call instance; level 4: four variables per call evaluated together)."""
    torch = torch_cuda()
    p = W.mlp_initial_params(5) + np.random.default_rng(6).normal(0, 0.1, mlp.N_PARAMS)
    M.mlmc_mlp_load(dev(p))
    q = mlp.deployed(p.astype(np.float32))
    n = 1000
    g = gpu_paths(W.GBM_CALL, level, n, M.MLMC_FP32, M.MLMC_RV_MLP, True, 1, 8)
    o = mlmc.level_paths(level, np.arange(n), W.GBM_CALL, rv_mode=mlmc.RV_MLP, precision=fp.FP32, nested=True,
                         kahan=True, seed=8, stream=1, mlp_params=q)
    assert np.max(np.abs(g["pf_hat"] - o["Pf_hat"])) <= 1e-13
    for key, ref in (("pf_bar", "Pf_bar"), ("pc_bar", "Pc_bar")):
        err = np.abs(g[key] - o[ref])
        assert np.all(err <= 1e-5 * np.maximum(np.abs(o[ref]), 1.0) + o[ref + "_allow"]), key
    # paths whose variables all round their second layer exactly meet the plain bar
    exact = (o["Pf_bar_allow"] == 0) & (o["Pc_bar_allow"] == 0)
    assert np.all(close(g["pf_bar"][exact], o["Pf_bar"][exact], 1e-5))


def test_full_size_sampled_mlp_paths_level10():
    """The learned variable's workload at full size: 2^22 paths at level 10 in the benchmark's
    launch, sampled paths against the oracle (binary32 bar plus the rounding allowance)."""
    torch = torch_cuda()
    p = W.mlp_initial_params(5) + np.random.default_rng(6).normal(0, 0.1, mlp.N_PARAMS)
    M.mlmc_mlp_load(dev(p))
    q = mlp.deployed(p.astype(np.float32))
    n, level = W.MLP_PATHS, 10
    g = gpu_paths(W.GBM_CALL, level, n, M.MLMC_FP32, M.MLMC_RV_MLP, True, 0, 0)
    idx = W.sampled_paths(n, 24)
    o = mlmc.level_paths(level, idx, W.GBM_CALL, rv_mode=mlmc.RV_MLP, precision=fp.FP32, nested=True,
                         kahan=False, seed=0, stream=1, mlp_params=q)
    assert np.max(np.abs(g["pf_hat"][idx] - o["Pf_hat"])) <= 1e-13 * max(1.0, np.max(np.abs(o["Pf_hat"])))
    for key, ref in (("pf_bar", "Pf_bar"), ("pc_bar", "Pc_bar")):
        err = np.abs(g[key][idx] - o[ref])
        assert np.all(err <= 1e-5 * np.maximum(np.abs(o[ref]), 1.0) + o[ref + "_allow"]), key


@pytest.fixture(scope="module")
def trained():
    torch = torch_cuda()
    params = dev(W.mlp_initial_params(0))
    hist = M.mlmc_mlp_train(M.mlp_cfg(), params)
    M.mlmc_mlp_load(params)
    return params, hist


def test_training_converges_and_beats_pwl(trained):
    _, hist = trained
    assert hist[-1] < hist[0] / 20
    x = np.arange(2 ** 20, dtype=np.uint64) * np.uint64(4096) + np.uint64(2047)
    z = icdf.exact(x)
    e_mlp = np.mean((gpu_icdf(x, M.MLMC_RV_MLP, M.MLMC_FP32) - z) ** 2)
    e_pwl = np.mean((icdf.approx(x, mlmc.RV_PWL, fp.FP32).astype(np.float64) - z) ** 2)
    assert e_mlp < e_pwl / 3, (e_mlp, e_pwl)


@pytest.mark.parametrize("level", [2, 6])
def test_four_way_variance_mlp_below_pwl(trained, level):
    n = 2 ** 18
    sde = M.gbm(payoff=M.MLMC_PAYOFF_CALL)
    v = {}
    for mode in (M.MLMC_NESTED_MLP, M.MLMC_NESTED_PWL16):
        r = M.mlmc_level(sde, level, n, M.MLMC_FP32, mode, 0, 0)
        v[mode] = E.level_stats(r["sum"][1], r["sumsq"][1], n)[1]
    assert v[M.MLMC_NESTED_MLP] < v[M.MLMC_NESTED_PWL16] / 2, v
