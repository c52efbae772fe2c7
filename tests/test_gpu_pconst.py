"""GPU parity of the piecewise-constant approximate variable (4096 equal cells, cell means of
Phi^{-1}) against the oracle: the variable bit for bit in every precision (a table lookup
and a sign), per-path payoffs bit for bit in binary32, binary16 and bfloat16 (the same
sequence of correctly rounded operations, no fitted arithmetic in the variable), the
binary64 exact pair and diagnostic within 1e-13, level sums within the per-path tolerances,
Milstein included, and the full-size level-10 launch on sampled paths."""

import numpy as np
import pytest

import mlmc_workloads as W
from gpu_util import gpu_icdf, gpu_paths
from oracle import fp, icdf, mlmc, philox
from test_gpu_parity import close, sums_close

import paper_2012_09739_amd as M

pytestmark = pytest.mark.gpu
PC = mlmc.RV_PCONST


@pytest.mark.parametrize("precision", [fp.FP64, fp.FP32, fp.FP16, fp.BF16])
def test_pconst_variable_bit_exact(precision):
    w = philox.words(5, 0, 3, 0, np.arange(8192, dtype=np.uint64), 8).ravel()
    edges = [0, 1, 2 ** 20 - 1, 2 ** 20, 2 ** 31 - 2 ** 20, 2 ** 31 - 1, 2 ** 31, 2 ** 32 - 2 ** 20, 2 ** 32 - 1]
    w = np.concatenate([w, np.array(edges, dtype=np.uint32)])
    got = gpu_icdf(w, M.MLMC_RV_PCONST4096, precision)
    want = fp.to64(icdf.approx(w, PC, precision))
    if precision == fp.FP64:   # the library's binary64 means (long double) within 1e-15 of the oracle's
        assert np.all(np.abs(got - want) <= 1e-15 * np.abs(want))
        np.testing.assert_array_equal(got, -gpu_icdf(np.uint32(2 ** 32 - 1) - w, M.MLMC_RV_PCONST4096, precision))
    else:
        np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("scheme", [M.MLMC_SCHEME_EM, M.MLMC_SCHEME_MILSTEIN])
@pytest.mark.parametrize("kahan", [0, 1])
@pytest.mark.parametrize("precision", [fp.FP32, fp.FP16, fp.BF16])
@pytest.mark.parametrize("level", [0, 1, 3, 6])
def test_nested_per_path_bit_exact(level, precision, kahan, scheme):
    n = 700
    sde = W.GBM_CALL
    g = gpu_paths(sde, level, n, precision, PC, True, kahan, 4, diag=True, scheme=scheme)
    o = mlmc.level_paths(level, np.arange(n), sde, rv_mode=PC, precision=precision, nested=True,
                         kahan=bool(kahan), seed=4, stream=1, diag=True, scheme=scheme)
    np.testing.assert_array_equal(g["pf_bar"], o["Pf_bar"])
    np.testing.assert_array_equal(g["pc_bar"], o["Pc_bar"])
    assert np.all(close(g["pf_hat"], o["Pf_hat"], 1e-13))
    assert np.all(close(g["pc_hat"], o["Pc_hat"], 1e-13))
    assert np.all(close(g["xf_tilde"], o["Xf_tilde"], 1e-13))


@pytest.mark.parametrize("level", [0, 2, 5])
def test_approx_fp64_per_path(level):
    n = 500
    g = gpu_paths(W.GBM, level, n, fp.FP64, PC, False, 0, 7)
    o = mlmc.level_paths(level, np.arange(n), W.GBM, rv_mode=PC, precision=fp.FP64, nested=False,
                         kahan=False, seed=7)
    assert np.all(close(g["pf_bar"], o["Pf_bar"], 1e-13))
    assert np.all(close(g["pc_bar"], o["Pc_bar"], 1e-13))


def test_nested_sums_match_oracle_terms():
    level, n = 4, 3000
    r = M.mlmc_level(M.gbm(payoff=M.MLMC_PAYOFF_CALL), level, n, M.MLMC_FP32, M.MLMC_NESTED_PCONST4096, 1, 8)
    o = mlmc.level_paths(level, np.arange(n), W.GBM_CALL, rv_mode=PC, precision=fp.FP32, nested=True,
                         kahan=True, seed=8, stream=1)
    for k in range(3):
        assert sums_close(r["sum"][k], r["sumsq"][k], o, k), k


def test_full_size_sampled_paths_level10():
    # the bench configuration's level-10 launch (2^20 paths), checked on sampled paths
    n, level = 1 << 20, 10
    idx = np.array([0, 1, 63, 64, 65, 4097, 123457, 524288, n - 65, n - 2, n - 1])
    g = gpu_paths(W.GBM_CALL, level, n, fp.FP32, PC, True, 1, 0)
    o = mlmc.level_paths(level, idx, W.GBM_CALL, rv_mode=PC, precision=fp.FP32, nested=True, kahan=True,
                         seed=0, stream=1)
    np.testing.assert_array_equal(g["pf_bar"][idx], o["Pf_bar"])
    np.testing.assert_array_equal(g["pc_bar"][idx], o["Pc_bar"])
    assert np.all(close(g["pf_hat"][idx], o["Pf_hat"], 1e-13))
    assert np.all(close(g["pc_hat"][idx], o["Pc_hat"], 1e-13))
