"""GPU tests of the single-level calls that run one eight-wave block per chunk (nested
binary32 and plain binary64, level >= 6, at most four partial rows per CU): their sums equal bit for bit those of
the single-wave code (a batch item with cooperative chunks switched off runs that code and the
same fixed-order reduction), and their terms match the per-path payoffs of the oracle."""

import numpy as np
import pytest
import torch  # noqa: F401

import mlmc_workloads as W
from gpu_util import gbm_struct, torch_cuda
from oracle import fp, mlmc
from test_gpu_parity import sums_close

import paper_2012_09739_amd as M

pytestmark = pytest.mark.gpu

MODES = {M.MLMC_RV_PWL16: M.MLMC_NESTED_PWL16, M.MLMC_RV_CUBIC16: M.MLMC_NESTED_CUBIC16}


def level_call(sde, level, n, rv, kahan, seed):
    torch = torch_cuda()
    args = M.level_args(gbm_struct(sde), level, n, M.MLMC_FP32, MODES[rv], kahan, seed)
    out = torch.zeros(8, dtype=torch.float64, device="cuda")
    M.mlmc_level_ex(args, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("rv", [M.MLMC_RV_PWL16, M.MLMC_RV_CUBIC16])
@pytest.mark.parametrize("kahan", [0, 1])
def test_cooperative_level_calls_equal_the_single_wave_code(rv, kahan):
    # levels 6..12 with ragged path counts (one to 1024 rows of 64 paths; level 6 ends on a
    # partial phase of 8 steps), against one batch whose items run the single-wave code
    # (coop_level 25: no cooperative chunks)
    torch = torch_cuda()
    sde = W.NESTED_FP32["sde"]
    cases = [(6, 129), (7, 4000), (8, 777), (8, 65536), (9, 64), (10, 1000), (11, 65), (12, 3000)]
    items = [M.item(gbm_struct(sde), l, n, M.MLMC_FP32, kahan, 4, pset=0, stream=1) for l, n in cases]
    out = torch.zeros((len(items), 8), dtype=torch.float64, device="cuda")
    plan = M.mlmc_batch_create(items, rv, out, M.mlmc_batch_cfg_t(16, 256, 25, 25, 8))
    try:
        M.mlmc_batch_run(plan)
        torch.cuda.synchronize()
        single_wave = out.cpu().numpy()
    finally:
        M.mlmc_batch_destroy(plan)
    for (l, n), want in zip(cases, single_wave):
        np.testing.assert_array_equal(level_call(sde, l, n, rv, kahan, 4), want, err_msg=str((l, n)))


@pytest.mark.parametrize("rv", [M.MLMC_RV_PWL16, M.MLMC_RV_CUBIC16])
@pytest.mark.parametrize("level,n", [(10, 200), (6, 129)])
def test_cooperative_level_sums_match_oracle(rv, level, n):
    # a few chunks, the last one ragged (level 6: 64 steps, two full phases and one of 8): the
    # two-way approximate, four-way and two-way exact sums against the oracle's per-path terms
    sde = W.NESTED_FP32["sde"]
    got = level_call(sde, level, n, rv, 1, 7)
    o = mlmc.level_paths(level, np.arange(n), sde, rv_mode=mlmc.RV_PWL if rv == M.MLMC_RV_PWL16 else mlmc.RV_CUBIC,
                         precision=fp.FP32, nested=True, kahan=True, seed=7, stream=1)
    for k in range(3):
        assert sums_close(got[k], got[4 + k], o, k), k


@pytest.mark.parametrize("prec,mode,kahan", [(M.MLMC_FP64, M.MLMC_EXACT, 0), (M.MLMC_FP32, M.MLMC_NESTED_PWL16, 1),
                                             (M.MLMC_FP32, M.MLMC_NESTED_CUBIC16, 0)])
@pytest.mark.parametrize("level", [6, 9])
def test_cooperative_partial_rows_equal_single_wave_rows(prec, mode, kahan, level):
    # 1024 rows of 64 paths (four per CU: cooperative) against 1025 rows (single-wave kernel):
    # the partial rows of the common paths, read back from the workspaces, agree bit for bit
    torch = torch_cuda()
    sde = gbm_struct(W.NESTED_FP32["sde"])
    # the library takes the cooperative kernel up to four partial rows per CU
    n_coop = 4 * torch.cuda.get_device_properties(0).multi_processor_count * 64
    rows = {}
    for n in (n_coop, n_coop + 64):
        args = M.level_args(sde, level, n, prec, mode, kahan, 11)
        nb = M.mlmc_level_workspace_bytes(args)
        ws = torch.full((nb // 8,), float("nan"), dtype=torch.float64, device="cuda")
        out = torch.zeros(8, dtype=torch.float64, device="cuda")
        M.mlmc_level_ex(args, out, ws, nb)
        torch.cuda.synchronize()
        rows[n] = ws[: (n // 64) * 8].cpu().numpy().reshape(-1, 8)
    np.testing.assert_array_equal(rows[n_coop], rows[n_coop + 64][: n_coop // 64])
    assert np.all(np.isfinite(rows[n_coop]))


@pytest.mark.parametrize("level,n", [(6, 1000), (7, 333)])
def test_cooperative_plain_fp64_sums_match_oracle(level, n):
    # the plain binary64 estimator through the cooperative kernel (at most four rows per CU)
    # against the oracle's per-path two-way terms
    sde = W.PLAIN_FP64["sde"]
    seed = W.PLAIN_FP64["seed"]
    r = M.mlmc_level(gbm_struct(sde), level, n, M.MLMC_FP64, M.MLMC_EXACT, 0, seed)
    o = mlmc.level_paths(level, np.arange(n), sde, rv_mode=mlmc.RV_EXACT, precision=fp.FP64, nested=False,
                         kahan=False, seed=seed)
    assert sums_close(r["sum"][0], r["sumsq"][0], o, 0)
    assert r["path_steps"] == n * 2 ** level
