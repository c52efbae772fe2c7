"""GPU parity of the Milstein level kernels against the oracle's Milstein scheme: the binary64
exact pair within 1e-13 (relative, per path), the binary16 and bfloat16 payoffs bit for bit
(the same sequence of correctly rounded operations), binary32 within 1e-5, level sums within
the per-path tolerances, and the exact level variances of the closed form (order 1)."""

import math

import numpy as np
import pytest

import mlmc_workloads as W
from gpu_util import gpu_paths
from milstein_closed_forms import level_moments
from oracle import fp, mlmc
from test_gpu_parity import close, sums_close

import paper_2012_09739_amd as M
from paper_2012_09739_amd import estimators as E

pytestmark = pytest.mark.gpu
MIL = M.MLMC_SCHEME_MILSTEIN


def _oracle(level, n, sde, **kw):
    return mlmc.level_paths(level, np.arange(n), sde, scheme=mlmc.SCHEME_MILSTEIN, **kw)


@pytest.mark.parametrize("level", [0, 1, 2, 3, 6])
def test_plain_fp64_per_path(level):
    n = 1000
    g = gpu_paths(W.GBM, level, n, M.MLMC_FP64, mlmc.RV_EXACT, False, 0, 3, scheme=MIL)
    o = _oracle(level, n, W.GBM, rv_mode=mlmc.RV_EXACT, precision=fp.FP64, nested=False, kahan=False, seed=3)
    assert np.all(close(g["pf_hat"], o["Pf_hat"], 1e-13))
    assert np.all(close(g["pc_hat"], o["Pc_hat"], 1e-13))


@pytest.mark.parametrize("kahan", [0, 1])
@pytest.mark.parametrize("rv", [mlmc.RV_PWL, mlmc.RV_CUBIC])
@pytest.mark.parametrize("precision", [fp.FP16, fp.BF16])
@pytest.mark.parametrize("level", [0, 1, 3, 6])
def test_nested_16bit_per_path_bit_exact(level, precision, rv, kahan):
    n = 700     # not a multiple of the chunk
    sde = W.GBM_CALL
    g = gpu_paths(sde, level, n, precision, rv, True, kahan, 4, diag=True, scheme=MIL)
    o = _oracle(level, n, sde, rv_mode=rv, precision=precision, nested=True, kahan=bool(kahan), seed=4,
                stream=1, diag=True)
    np.testing.assert_array_equal(g["pf_bar"], o["Pf_bar"])
    np.testing.assert_array_equal(g["pc_bar"], o["Pc_bar"])
    assert np.all(close(g["pf_hat"], o["Pf_hat"], 1e-13))
    assert np.all(close(g["pc_hat"], o["Pc_hat"], 1e-13))
    assert np.all(close(g["xf_tilde"], o["Xf_tilde"], 1e-13))


@pytest.mark.parametrize("kahan", [0, 1])
@pytest.mark.parametrize("level", [0, 2, 5, 8])
def test_nested_fp32_per_path(level, kahan):
    n = 500
    g = gpu_paths(W.GBM_CALL, level, n, M.MLMC_FP32, mlmc.RV_PWL, True, kahan, 6, diag=True, scheme=MIL)
    o = _oracle(level, n, W.GBM_CALL, rv_mode=mlmc.RV_PWL, precision=fp.FP32, nested=True, kahan=bool(kahan),
                seed=6, stream=1, diag=True)
    assert np.all(close(g["pf_hat"], o["Pf_hat"], 1e-13))
    assert np.all(close(g["pf_bar"], o["Pf_bar"], 1e-5))
    assert np.all(close(g["pc_bar"], o["Pc_bar"], 1e-5))
    assert np.all(close(g["xf_tilde"], o["Xf_tilde"], 1e-13))


def test_nested_sums_match_oracle_terms():
    level, n = 4, 3000
    sde = W.GBM_CALL
    torch = pytest.importorskip("torch")
    args = M.level_args(M.gbm(payoff=M.MLMC_PAYOFF_CALL), level, n, M.MLMC_FP16, M.MLMC_NESTED_CUBIC16, 1, 8,
                        diag=1, scheme=MIL)
    out = torch.zeros(8, dtype=torch.float64, device="cuda")
    M.mlmc_level_ex(args, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    o = _oracle(level, n, sde, rv_mode=mlmc.RV_CUBIC, precision=fp.FP16, nested=True, kahan=True, seed=8,
                stream=1, diag=True)
    for k in range(4):
        assert sums_close(got[k], got[4 + k], o, k), k


@pytest.mark.parametrize("level", [2, 5, 8])
def test_plain_fp64_variance_matches_closed_form(level):
    # 2^20 paths: the sample variance of the level difference is within 2% of the exact one
    torch = pytest.importorskip("torch")
    m = 1 << 20
    args = M.level_args(M.gbm(), level, m, M.MLMC_FP64, M.MLMC_EXACT, 0, 12, scheme=MIL)
    out = torch.zeros(8, dtype=torch.float64, device="cuda")
    M.mlmc_level_ex(args, out)
    torch.cuda.synchronize()
    s = out.cpu().numpy()
    mean, var = E.level_stats(s[0], s[4], m)
    cf = level_moments(level)
    assert abs(var / float(cf["var"]) - 1) < 0.02
    assert abs(mean - float(cf["mean"])) < 4.5 * math.sqrt(float(cf["var"]) / m)
