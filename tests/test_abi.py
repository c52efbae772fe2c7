"""CPU tests of the C-ABI library: it loads, exports every entry point include/mlmc.h
declares, validates arguments before touching HIP, reports ENODEV without a GPU, and its
host-built coefficient tables agree with the oracle's (an independent construction)."""

import ctypes
import os
import re

import numpy as np
import pytest

import paper_2012_09739_amd as M
from oracle import fp, tables

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "mlmc.h")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(mlmc_\w+)\s*\(", text, re.M)))


def test_header_declares_entry_points():
    names = declared()
    for n in ("mlmc_level", "mlmc_level_ex", "mlmc_paths", "mlmc_uniforms", "mlmc_icdf", "mlmc_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(M.mlmc.LIB_PATH)
    for name in declared():
        assert hasattr(lib, name), name
    assert set(declared()) <= set(M.exported_symbols())


def _gpu_visible():
    try:
        import torch
        return torch.cuda.device_count() > 0
    except Exception:
        return False


@pytest.mark.parametrize("kw,code", [
    (dict(level=-1), M.MLMC_EINVAL), (dict(level=25), M.MLMC_EINVAL), (dict(precision=4), M.MLMC_EINVAL),
    (dict(precision=M.MLMC_BF16), M.MLMC_EINVAL), (dict(precision=M.MLMC_BF16, rv_mode=M.MLMC_NESTED_MLP), M.MLMC_EINVAL),
    (dict(rv_mode=-1), M.MLMC_EINVAL), (dict(rv_mode=9), M.MLMC_EINVAL), (dict(kahan=2), M.MLMC_EINVAL),
    (dict(precision=M.MLMC_FP32, rv_mode=M.MLMC_EXACT), M.MLMC_EINVAL), (dict(n_paths=2 ** 32 + 1), M.MLMC_EINVAL)])
def test_invalid_arguments(kw, code):
    a = dict(level=3, n_paths=10, precision=M.MLMC_FP64, rv_mode=M.MLMC_EXACT, kahan=0)
    a.update(kw)
    with pytest.raises(M.MlmcError) as e:
        M.mlmc_level(M.gbm(), a["level"], a["n_paths"], a["precision"], a["rv_mode"], a["kahan"], 0)
    assert e.value.code == code
    assert M.mlmc_last_error()


@pytest.mark.parametrize("rv_mode,scheme", [(M.MLMC_NESTED_MLP, M.MLMC_SCHEME_MILSTEIN), (M.MLMC_APPROX_MLP, 1),
                                            (M.MLMC_NESTED_PWL16, 2), (M.MLMC_EXACT, 7)])
def test_invalid_scheme(rv_mode, scheme):
    precision = M.MLMC_FP64 if rv_mode == M.MLMC_EXACT else M.MLMC_FP32
    a = M.level_args(M.gbm(), 3, 64, precision, rv_mode, 0, 0, scheme=scheme)
    assert M.mlmc_level_workspace_bytes(a) == 0
    assert M.lib().mlmc_paths(ctypes.byref(a), None, None, None, None, None, None) == M.MLMC_EINVAL
    assert "scheme" in M.mlmc_last_error().lower() or "milstein" in M.mlmc_last_error().lower()


@pytest.mark.parametrize("sde", [M.gbm(T=0.0), M.gbm(sigma=-1.0), M.gbm(payoff=7), M.gbm(mu=float("nan"))])
def test_invalid_sde(sde):
    with pytest.raises(M.MlmcError) as e:
        M.mlmc_level(sde, 3, 10, M.MLMC_FP64, M.MLMC_EXACT, 0, 0)
    assert e.value.code == M.MLMC_EINVAL


def test_null_pointers_rejected():
    lib = M.lib()
    r = M.mlmc_result_t()
    assert lib.mlmc_level(None, 1, 1, 0, 0, 0, 0, ctypes.byref(r)) == M.MLMC_EINVAL
    s = M.gbm()
    assert lib.mlmc_level(ctypes.byref(s), 1, 1, 0, 0, 0, 0, None) == M.MLMC_EINVAL
    args = M.level_args(s, 2, 10, 0, 0)
    assert lib.mlmc_level_ex(ctypes.byref(args), None, None, 0, None) == M.MLMC_EINVAL
    assert lib.mlmc_level_ex(None, None, None, 0, None) == M.MLMC_EINVAL
    assert lib.mlmc_table(1, 0, None) == M.MLMC_EINVAL
    assert lib.mlmc_level_workspace_bytes(None) == 0
    assert lib.mlmc_level_noalloc(ctypes.byref(args), None, None) == M.MLMC_EINVAL
    assert lib.mlmc_level_noalloc(None, None, None) == M.MLMC_EINVAL


@pytest.mark.parametrize("prec,n", [(M.MLMC_FP32, (1 << 22) + 1), (M.MLMC_FP64, 1 << 23),
                                    (M.MLMC_FP16, (1 << 23) + 1)])
def test_noalloc_size_limit_before_device(prec, n):
    # the fixed scratch holds 65536 chunks: 2^22 paths (2^23 in binary16); checked before any HIP call
    args = M.level_args(M.gbm(), 3, n, prec, M.MLMC_NESTED_PWL16)
    with pytest.raises(M.MlmcError) as e:
        M.mlmc_level_noalloc(args, 1 << 20, stream=0)
    assert e.value.code == M.MLMC_EINVAL
    assert "65536" in M.mlmc_last_error()


def test_workspace_size():
    # chunk partials (8 doubles per chunk), 128 stage rows of the reduction, 64 bytes of slack
    args = M.level_args(M.gbm(), 5, 1000, M.MLMC_FP32, M.MLMC_NESTED_PWL16)
    assert M.mlmc_level_workspace_bytes(args) == (16 + 128) * 8 * 8 + 64     # 16 chunks of 64 paths
    args16 = M.level_args(M.gbm(), 5, 1000, M.MLMC_FP16, M.MLMC_NESTED_PWL16)
    assert M.mlmc_level_workspace_bytes(args16) == (8 + 128) * 8 * 8 + 64    # 8 chunks of 128 paths
    # approximate-only estimators group 8, 4, 2 chunks per row at levels 2, 3, 4, one above
    for level, rows in ((2, 2), (3, 4), (4, 8), (5, 16)):
        a = M.level_args(M.gbm(), level, 1000, M.MLMC_FP32, M.MLMC_APPROX_PWL16)
        assert M.mlmc_level_workspace_bytes(a) == (rows + 128) * 8 * 8 + 64, level
    # levels 0 and 1 take 8 and 4 chunks per row for every estimator
    for prec, mode in ((M.MLMC_FP64, M.MLMC_EXACT), (M.MLMC_FP32, M.MLMC_APPROX_PWL16),
                       (M.MLMC_FP32, M.MLMC_NESTED_PWL16)):
        a = M.level_args(M.gbm(), 1, 1000, prec, mode)
        assert M.mlmc_level_workspace_bytes(a) == (4 + 128) * 8 * 8 + 64, mode


@pytest.mark.skipif(_gpu_visible(), reason="a GPU is visible")
def test_no_device_is_reported():
    with pytest.raises(M.MlmcError) as e:
        M.mlmc_level(M.gbm(), 3, 10, M.MLMC_FP64, M.MLMC_EXACT, 0, 0)
    assert e.value.code == M.MLMC_ENODEV


@pytest.mark.parametrize("rv,deg", [(M.MLMC_RV_PWL16, 1), (M.MLMC_RV_CUBIC16, 3)])
def test_library_table_matches_oracle_table(rv, deg):
    want = np.array(tables.table(deg))
    got = np.array(M.mlmc_table(rv, M.MLMC_FP64))
    assert np.all(got[:, deg + 1:] == 0)
    got = got[:, :deg + 1]
    assert np.max(np.abs(got - want) / np.abs(want)) < 1e-12
    for p, dt in ((M.MLMC_FP32, np.float32), (M.MLMC_FP16, np.float16)):
        np.testing.assert_array_equal(np.array(M.mlmc_table(rv, p))[:, :deg + 1], want.astype(dt).astype(np.float64))
    # bfloat16: one rounding of the binary64 coefficients to 8 significant bits
    np.testing.assert_array_equal(np.array(M.mlmc_table(rv, M.MLMC_BF16))[:, :deg + 1], fp.round_bits(want, 8))


def test_library_pconst_table_matches_oracle():
    want = np.array(tables.pconst())
    got = np.array(M.mlmc_pconst_table(M.MLMC_FP64))
    assert got.shape == (2048,)
    assert np.max(np.abs(got - want) / np.abs(want)) < 1e-15
    for p, prec in ((M.MLMC_FP32, fp.FP32), (M.MLMC_FP16, fp.FP16), (M.MLMC_BF16, fp.BF16)):
        np.testing.assert_array_equal(np.array(M.mlmc_pconst_table(p)), fp.to64(fp.rn(prec, want)))


def test_batch_validation_before_device():
    s = M.gbm()
    for bad in (M.item(s, -1, 10, M.MLMC_FP32), M.item(s, 3, 0, M.MLMC_FP32), M.item(s, 3, 10, M.MLMC_FP64),
                M.item(s, 3, 10, M.MLMC_FP16, kahan=3), M.item(M.gbm(T=-1.0), 3, 10, M.MLMC_FP32)):
        with pytest.raises(M.MlmcError) as e:
            M.mlmc_batch_create([bad], M.MLMC_RV_PWL16, 1)
        assert e.value.code == M.MLMC_EINVAL
    with pytest.raises(M.MlmcError) as e:
        M.mlmc_batch_create([M.item(s, 3, 10, M.MLMC_FP32)], M.MLMC_RV_EXACT, 1)
    assert e.value.code == M.MLMC_EINVAL
    for cfg in (M.mlmc_batch_cfg_t(16, 256, 25, 1), M.mlmc_batch_cfg_t(16, 256, 25, 26),
                M.mlmc_batch_cfg_t(3, 256, 25, 13), M.mlmc_batch_cfg_t(16, 256, 26, 13),
                M.mlmc_batch_cfg_t(16, 256, 25, 13, 6), M.mlmc_batch_cfg_t(4, 256, 25, 13, 8)):
        with pytest.raises(M.MlmcError) as e:
            M.mlmc_batch_create([M.item(s, 3, 10, M.MLMC_FP32)], M.MLMC_RV_PWL16, 1, cfg)
        assert e.value.code == M.MLMC_EINVAL
    assert M.lib().mlmc_batch_destroy(None) == M.MLMC_OK


def test_level_set_validation_before_device():
    lib = M.lib()
    good = M.level_args(M.gbm(), 3, 100, M.MLMC_FP32, M.MLMC_NESTED_PWL16)
    bad = M.level_args(M.gbm(), 3, 100, M.MLMC_FP32, M.MLMC_EXACT)  # the plain estimator is binary64
    res = (M.mlmc_result_t * 2)()
    arr = (M.mlmc_level_args_t * 2)(good, bad)
    assert lib.mlmc_level_set_run(arr, 2, res, None) == M.MLMC_EINVAL
    assert "call 1" in M.mlmc_last_error()
    assert lib.mlmc_level_set_run(arr, 0, res, None) == M.MLMC_EINVAL
    assert lib.mlmc_level_set_run(arr, 4097, res, None) == M.MLMC_EINVAL
    assert lib.mlmc_level_set_run(None, 1, res, None) == M.MLMC_EINVAL
    assert lib.mlmc_level_set_run(arr, 1, None, None) == M.MLMC_EINVAL


def test_uniforms_reject_more_steps_than_a_coarse_level_has():
    # levels 0 and 1 share each Philox call between paths: at most 2^level words per path
    lib = M.lib()
    for level, n_steps in ((0, 2), (1, 3)):
        assert lib.mlmc_uniforms(0, 0, level, 0, 0, 0, n_steps, None, None) == M.MLMC_EINVAL
        assert "steps" in M.mlmc_last_error()
