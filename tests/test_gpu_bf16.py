"""GPU parity of the emulated bfloat16 paths (8 significant bits, round to nearest even after
every operation) against the oracle's bfloat16 emulation: the approximate variables and the
low-precision payoffs bit for bit (the same sequence of correctly rounded operations), the
binary64 exact pair and diagnostic path within 1e-13, the level sums within the per-path
tolerances, and the rounding-difference variance under B_l with rho = 2^-8."""

import math

import numpy as np
import pytest

import mlmc_workloads as W
from gpu_util import gpu_icdf, gpu_paths
from oracle import fp, icdf, mlmc, philox
from test_gpu_parity import close, sums_close

import paper_2012_09739_amd as M
from paper_2012_09739_amd import estimators as E

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("rv", [mlmc.RV_PWL, mlmc.RV_CUBIC])
def test_bf16_approximate_variable_bit_exact(rv):
    w = philox.words(5, 0, 3, 0, np.arange(4096, dtype=np.uint64), 8).ravel()
    w = np.concatenate([w, np.array([0, 1, 2 ** 31 - 1, 2 ** 31, 2 ** 32 - 1, 65535, 65536], dtype=np.uint32)])
    got = gpu_icdf(w, rv, M.MLMC_BF16)
    want = fp.to64(icdf.approx(w, rv, fp.BF16))
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("kahan", [0, 1])
@pytest.mark.parametrize("rv", [mlmc.RV_PWL, mlmc.RV_CUBIC])
@pytest.mark.parametrize("level", [0, 1, 3, 6])
def test_nested_bf16_per_path(level, rv, kahan):
    n = 700     # not a multiple of the 64-path chunk
    sde = W.GBM_CALL
    g = gpu_paths(sde, level, n, M.MLMC_BF16, rv, True, kahan, 4, diag=True)
    o = mlmc.level_paths(level, np.arange(n), sde, rv_mode=rv, precision=fp.BF16, nested=True,
                         kahan=bool(kahan), seed=4, stream=1, diag=True)
    np.testing.assert_array_equal(g["pf_bar"], o["Pf_bar"])
    np.testing.assert_array_equal(g["pc_bar"], o["Pc_bar"])
    assert np.all(close(g["pf_hat"], o["Pf_hat"], 1e-13))
    assert np.all(close(g["xf_tilde"], o["Xf_tilde"], 1e-13))


def test_bf16_level_sums_and_rounding_bound():
    level, n = 5, 4000
    sde = W.GBM
    r = M.mlmc_level(M.gbm(), level, n, M.MLMC_BF16, M.MLMC_APPROX_CUBIC16, 0, 9)
    o = mlmc.level_paths(level, np.arange(n), sde, rv_mode=mlmc.RV_CUBIC, precision=fp.BF16, nested=False,
                         kahan=False, seed=9)
    assert sums_close(r["sum"][0], r["sumsq"][0], o, 0)
    # rounding-difference variance of the binary16-width sweep's bfloat16 end, under B_l
    args = M.level_args(M.gbm(), level, 1 << 16, M.MLMC_BF16, M.MLMC_APPROX_CUBIC16, 0, 9, diag=1)
    import torch
    out = torch.zeros(8, dtype=torch.float64, device="cuda")
    M.mlmc_level_ex(args, out)
    torch.cuda.synchronize()
    s = out.cpu().numpy()
    var = E.level_stats(s[3], s[7], 1 << 16)[1]
    N, rho = 2 ** level, fp.UNIT_ROUNDOFF[fp.BF16]
    bound = N * rho * rho * (1 + 0.05 / N) ** (2 * N) * math.exp(0.04) * math.exp(2 * 0.05 + 0.04)
    assert 0 < var <= bound
