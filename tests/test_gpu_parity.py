"""GPU parity: the HIP path through the C-ABI against the CPU oracle, element by element.

Bars: uniform words bit-exact; binary64 per-path payoffs within 1e-13 relative;
binary32 per-path payoffs within 1e-5 relative (|d| <= 1e-5 max(|o|, 1)); binary16 per-path
values equal to the oracle's per-operation emulation (the arithmetic is the same sequence
of correctly rounded operations), with the statistical checks in test_gpu_stats; level
sums within 1e-12 of sum |x| (reduction order differs from the oracle's exact sum).
"""

import math

import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection: the first import can take a minute)

import mlmc_workloads as W
from gpu_util import gpu_icdf, gpu_paths, gpu_uniforms, torch_cuda
from oracle import fp, icdf, mlmc, philox

import paper_2012_09739_amd as M
from paper_2012_09739_amd import estimators as E

pytestmark = pytest.mark.gpu

rng = np.random.default_rng(11)
WORDS = np.concatenate([np.array([0, 1, 2, 3, 2 ** 15, 2 ** 16 - 1, 2 ** 16, 2 ** 31 - 1, 2 ** 31, 2 ** 31 + 1,
                                  2 ** 32 - 2, 2 ** 32 - 1], dtype=np.uint64),
                        rng.integers(0, 2 ** 32, 20000, dtype=np.uint64),
                        (2.0 ** rng.uniform(0, 32, 5000)).astype(np.uint64)])


def close(got, want, rtol):
    return np.abs(got - want) <= rtol * np.maximum(np.abs(want), 1.0)


def sums_close(got_sum, got_sq, o, k):
    """Level sums of term k against the oracle's exactly rounded sums.  Terms built from
    binary64 paths inherit their 1e-13 per-path tolerance (inverse CDF and binary64 table
    differ in the last bits), the rest only the reduction's rounding."""
    t = o["terms"][k]
    per_path = 1e-12 * np.abs(t)
    if k in (1, 2) or "Pf_bar" not in o:
        per_path = per_path + 1e-13 * (np.abs(o["Pf_hat"]) + np.abs(o["Pc_hat"]))
    if k == 3:   # binary64 path with the library's own binary64 table (1e-13 per path)
        per_path = per_path + 1e-13 * np.abs(o["Xf_tilde"])
    ok_sum = abs(got_sum - math.fsum(t)) <= per_path.sum() + 1e-300
    ok_sq = abs(got_sq - math.fsum(t * t)) <= (2 * np.abs(t) * per_path + 1e-12 * t * t).sum() + 1e-300
    return ok_sum and ok_sq


@pytest.mark.parametrize("seed,stream,level,pset,path0,n_paths,n_steps", [
    (0, 0, 3, 0, 0, 100, 8), (0x0123456789ABCDEF, 1, 10, 7, 12345, 37, 1024),
    (5, 65535, 0, 2 ** 32 - 1, 2 ** 32 - 5, 5, 1), (9, 3, 1, 0, 1000, 64, 2), (1, 2, 14, 63, 0, 3, 13)])
def test_uniforms_bit_exact(seed, stream, level, pset, path0, n_paths, n_steps):
    got = gpu_uniforms(seed, stream, level, pset, path0, n_paths, n_steps)
    want = philox.words(seed, stream, level, pset, np.arange(path0, path0 + n_paths), n_steps)
    np.testing.assert_array_equal(got, want)


def test_icdf_exact_fp64():
    got = gpu_icdf(WORDS, M.MLMC_RV_EXACT, M.MLMC_FP64)
    want = icdf.exact(WORDS)
    rel = np.abs(got - want) / np.abs(want)
    assert rel.max() < 1e-14, rel.max()
    # exactly odd under the mirror word
    np.testing.assert_array_equal(gpu_icdf(np.uint64(2 ** 32 - 1) - WORDS, M.MLMC_RV_EXACT, M.MLMC_FP64), -got)


@pytest.mark.parametrize("rv", [M.MLMC_RV_PWL16, M.MLMC_RV_CUBIC16])
@pytest.mark.parametrize("precision", [M.MLMC_FP64, M.MLMC_FP32, M.MLMC_FP16])
def test_icdf_dyadic(rv, precision):
    got = gpu_icdf(WORDS, rv, precision)
    want = icdf.approx(WORDS, rv, precision).astype(np.float64)
    if precision == M.MLMC_FP64:
        # the library's binary64 table is its own L2 fit; agrees with the oracle's to 1e-13
        assert np.all(close(got, want, 1e-13))
    else:
        np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("level", W.PLAIN_FP64["levels"])
def test_plain_fp64_per_path(level):
    n = W.PLAIN_FP64["n_paths"]
    sde = W.PLAIN_FP64["sde"]
    g = gpu_paths(sde, level, n, M.MLMC_FP64, 0, False, 0, W.PLAIN_FP64["seed"])
    o = mlmc.level_paths(level, np.arange(n), sde, rv_mode=0, precision=fp.FP64, nested=False, kahan=False,
                         seed=W.PLAIN_FP64["seed"])
    assert np.all(close(g["pf_hat"], o["Pf_hat"], 1e-13))
    assert np.all(close(g["pc_hat"], o["Pc_hat"], 1e-13))
    if level == 0:
        assert np.all(g["pc_hat"] == 0)


@pytest.mark.parametrize("level", W.PLAIN_FP64["levels"])
def test_plain_fp64_level_sums(level):
    n = W.PLAIN_FP64["n_paths"]
    sde = W.PLAIN_FP64["sde"]
    r = M.mlmc_level(M.gbm(**{k: sde[k] for k in ("mu", "sigma", "x0", "T", "payoff", "strike")}), level, n,
                     M.MLMC_FP64, M.MLMC_EXACT, 0, W.PLAIN_FP64["seed"])
    o = mlmc.level_paths(level, np.arange(n), sde, rv_mode=0, precision=fp.FP64, nested=False, kahan=False,
                         seed=W.PLAIN_FP64["seed"])
    assert sums_close(r["sum"][0], r["sumsq"][0], o, 0)
    assert all(math.isnan(r["sum"][k]) for k in (1, 2, 3))
    assert r["path_steps"] == n * 2 ** level and r["cost_seconds"] > 0


@pytest.mark.parametrize("kahan", [0, 1])
@pytest.mark.parametrize("level", [0, 1, 2, 5, 10])
def test_nested_fp32_pwl_per_path(level, kahan):
    n = 2000 if level < 10 else 500
    sde = W.NESTED_FP32["sde"]
    g = gpu_paths(sde, level, n, M.MLMC_FP32, M.MLMC_RV_PWL16, True, kahan, 0, diag=True)
    o = mlmc.level_paths(level, np.arange(n), sde, rv_mode=mlmc.RV_PWL, precision=fp.FP32, nested=True,
                         kahan=bool(kahan), seed=0, stream=1, diag=True)
    assert np.all(close(g["pf_hat"], o["Pf_hat"], 1e-13))
    assert np.all(close(g["pc_hat"], o["Pc_hat"], 1e-13))
    assert np.all(close(g["pf_bar"], o["Pf_bar"], 1e-5))
    assert np.all(close(g["pc_bar"], o["Pc_bar"], 1e-5))
    assert np.all(close(g["xf_tilde"], o["Xf_tilde"], 1e-13))
    # same sequence of correctly rounded binary32 operations: expected bit-identical
    assert np.mean(g["pf_bar"] == o["Pf_bar"]) == 1.0


@pytest.mark.parametrize("kahan", [0, 1])
@pytest.mark.parametrize("rv", [mlmc.RV_PWL, mlmc.RV_CUBIC])
@pytest.mark.parametrize("level", [0, 1, 3, 6])
def test_nested_fp16_per_path(level, rv, kahan):
    n = 1000   # not a multiple of the 128-path chunk: exercises the ragged tail
    sde = W.NESTED_FP16["sde"]
    g = gpu_paths(sde, level, n, M.MLMC_FP16, rv, True, kahan, 3, diag=True)
    o = mlmc.level_paths(level, np.arange(n), sde, rv_mode=rv, precision=fp.FP16, nested=True,
                         kahan=bool(kahan), seed=3, stream=1, diag=True)
    assert np.all(close(g["pf_hat"], o["Pf_hat"], 1e-13))
    np.testing.assert_array_equal(g["pf_bar"], o["Pf_bar"])
    np.testing.assert_array_equal(g["pc_bar"], o["Pc_bar"])
    assert np.all(close(g["xf_tilde"], o["Xf_tilde"], 1e-13))


@pytest.mark.parametrize("offset", [0, 1, 2, 3, 2 ** 32 - 1003])
@pytest.mark.parametrize("level", [0, 1])
def test_coarse_levels_share_calls_at_any_path_offset(level, offset):
    """Levels 0 and 1 draw one Philox call per 4 / 2^l consecutive paths; a slice that starts
    inside a group (offset not a multiple of the group) takes the words of two calls per lane.
    Nested binary32 (Kahan) and packed binary16 paths and the plain binary64 ones, per path, with
    a ragged count, against the oracle's words of the same global paths."""
    n = 1000
    sde = W.NESTED_FP32["sde"]
    paths = np.arange(offset, offset + n)
    g = gpu_paths(sde, level, n, M.MLMC_FP32, M.MLMC_RV_PWL16, True, 1, 5, path_offset=offset)
    o = mlmc.level_paths(level, paths, sde, rv_mode=mlmc.RV_PWL, precision=fp.FP32, nested=True, kahan=True,
                         seed=5, stream=1)
    assert np.all(close(g["pf_hat"], o["Pf_hat"], 1e-13))
    np.testing.assert_array_equal(g["pf_bar"], o["Pf_bar"])     # binary32 emulated exactly
    np.testing.assert_array_equal(g["pc_bar"], o["Pc_bar"])
    g16 = gpu_paths(sde, level, n, M.MLMC_FP16, mlmc.RV_CUBIC, True, 1, 5, path_offset=offset)
    o16 = mlmc.level_paths(level, paths, sde, rv_mode=mlmc.RV_CUBIC, precision=fp.FP16, nested=True, kahan=True,
                           seed=5, stream=1)
    np.testing.assert_array_equal(g16["pf_bar"], o16["Pf_bar"])
    np.testing.assert_array_equal(g16["pc_bar"], o16["Pc_bar"])
    assert np.all(close(g16["pf_hat"], o16["Pf_hat"], 1e-13))
    g64 = gpu_paths(sde, level, n, M.MLMC_FP64, 0, False, 0, 5, path_offset=offset)
    o64 = mlmc.level_paths(level, paths, sde, rv_mode=0, precision=fp.FP64, nested=False, kahan=False, seed=5)
    assert np.all(close(g64["pf_hat"], o64["Pf_hat"], 1e-13))
    assert np.all(close(g64["pc_hat"], o64["Pc_hat"], 1e-13))


@pytest.mark.parametrize("level", [0, 1])
def test_approx_only_coarse_levels_per_path(level):
    # every variant runs levels 0 and 1 through the shared-call instance, the approximate-only
    # ones included
    n = 777
    sde = W.GBM
    for precision, rv in ((M.MLMC_FP32, mlmc.RV_PWL), (M.MLMC_FP16, mlmc.RV_CUBIC)):
        g = gpu_paths(sde, level, n, precision, rv, False, 1, 17, path_offset=6)
        o = mlmc.level_paths(level, np.arange(6, 6 + n), sde, rv_mode=rv, precision=precision, nested=False,
                             kahan=True, seed=17)
        np.testing.assert_array_equal(g["pf_bar"], o["Pf_bar"])
        np.testing.assert_array_equal(g["pc_bar"], o["Pc_bar"])
        assert np.all(np.isnan(g["pf_hat"]))


@pytest.mark.parametrize("precision,rv", [(M.MLMC_FP64, mlmc.RV_PWL), (M.MLMC_FP64, mlmc.RV_CUBIC),
                                          (M.MLMC_FP32, mlmc.RV_CUBIC)])
def test_approx_only_per_path(precision, rv):
    n, level = 777, 4
    sde = W.GBM
    g = gpu_paths(sde, level, n, precision, rv, False, 1, 17)
    o = mlmc.level_paths(level, np.arange(n), sde, rv_mode=rv, precision=precision, nested=False, kahan=True,
                         seed=17)
    tol = 1e-13 if precision == M.MLMC_FP64 else 1e-5
    assert np.all(close(g["pf_bar"], o["Pf_bar"], tol))
    assert np.all(np.isnan(g["pf_hat"]))   # the exact pair is not computed


def test_nested_sums_match_oracle_terms():
    n, level = 3000, 4
    sde = W.GBM_CALL
    args = M.level_args(M.gbm(payoff=1), level, n, M.MLMC_FP32, M.MLMC_NESTED_PWL16, 1, 0, diag=1)
    torch = torch_cuda()
    out = torch.zeros(8, dtype=torch.float64, device="cuda")
    M.mlmc_level_ex(args, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    o = mlmc.level_paths(level, np.arange(n), sde, rv_mode=mlmc.RV_PWL, precision=fp.FP32, nested=True,
                         kahan=True, seed=0, stream=1, diag=True)
    for k in range(4):
        assert sums_close(got[k], got[4 + k], o, k), k


@pytest.mark.parametrize("precision,rv,kahan", [(M.MLMC_FP32, mlmc.RV_PWL, 0), (M.MLMC_FP32, mlmc.RV_PWL, 1),
                                                (M.MLMC_FP16, mlmc.RV_CUBIC, 1)])
@pytest.mark.parametrize("level,n", [(2, 3001), (3, 1999), (4, 1000), (5, 777)])
def test_approximate_sums_match_oracle_terms(level, n, precision, rv, kahan):
    """Two-way approximate estimators, whose partial rows hold 8, 4, 2 chunks at levels 2, 3, 4
    (one above): the sums against the oracle's per-path terms, ragged last rows included."""
    sde = W.GBM_CALL
    mode = M.MLMC_APPROX_PWL16 if rv == mlmc.RV_PWL else M.MLMC_APPROX_CUBIC16
    args = M.level_args(M.gbm(payoff=1), level, n, precision, mode, kahan, 6)
    torch = torch_cuda()
    out = torch.zeros(8, dtype=torch.float64, device="cuda")
    M.mlmc_level_ex(args, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    o = mlmc.level_paths(level, np.arange(n), sde, rv_mode=rv, precision=fp.FP32 if precision == M.MLMC_FP32 else fp.FP16,
                         nested=False, kahan=bool(kahan), seed=6, stream=0)
    assert sums_close(got[0], got[4], o, 0)
    assert got[1] == 0 and got[2] == 0 and got[5] == 0 and got[6] == 0


def test_full_size_sampled_paths_nested_fp32():
    """2^20 paths at level 10 in the benchmark's launch; oracle recomputes sampled paths."""
    n, level = W.NESTED_FP32["n_paths"], 10
    sde = W.NESTED_FP32["sde"]
    g = gpu_paths(sde, level, n, M.MLMC_FP32, M.MLMC_RV_PWL16, True, 1, 0)
    idx = W.sampled_paths(n, 48)
    o = mlmc.level_paths(level, idx, sde, rv_mode=mlmc.RV_PWL, precision=fp.FP32, nested=True, kahan=True,
                         seed=0, stream=1)
    assert np.all(close(g["pf_hat"][idx], o["Pf_hat"], 1e-13))
    assert np.all(close(g["pf_bar"][idx], o["Pf_bar"], 1e-5))
    assert np.all(close(g["pc_bar"][idx], o["Pc_bar"], 1e-5))


def test_full_size_sampled_paths_fp16():
    n, level = W.NESTED_FP16["n_paths"], 6
    sde = W.NESTED_FP16["sde"]
    g = gpu_paths(sde, level, n, M.MLMC_FP16, M.MLMC_RV_CUBIC16, True, 1, 0, diag=True)
    idx = W.sampled_paths(n, 48)
    o = mlmc.level_paths(level, idx, sde, rv_mode=mlmc.RV_CUBIC, precision=fp.FP16, nested=True, kahan=True,
                         seed=0, stream=1, diag=True)
    np.testing.assert_array_equal(g["pf_bar"][idx], o["Pf_bar"])
    assert np.all(close(g["pf_hat"][idx], o["Pf_hat"], 1e-13))


@pytest.mark.parametrize("level", [0, 1])
def test_full_size_sampled_paths_coarse_levels(level):
    """The benchmark's coarse levels at full size (shared Philox calls): binary32 nested at 2^20
    paths and packed binary16 nested at 2^24, sampled paths (the ends of the range included)."""
    for precision, rv, n in ((M.MLMC_FP32, mlmc.RV_PWL, W.NESTED_FP32["n_paths"]),
                             (M.MLMC_FP16, mlmc.RV_CUBIC, W.NESTED_FP16["n_paths"])):
        sde = W.NESTED_FP32["sde"]
        g = gpu_paths(sde, level, n, precision, rv, True, 1, 0)
        idx = W.sampled_paths(n, 48)
        o = mlmc.level_paths(level, idx, sde, rv_mode=rv, precision=fp.FP32 if precision == M.MLMC_FP32 else fp.FP16,
                             nested=True, kahan=True, seed=0, stream=1)
        assert np.all(close(g["pf_hat"][idx], o["Pf_hat"], 1e-13))
        np.testing.assert_array_equal(g["pf_bar"][idx], o["Pf_bar"])
        np.testing.assert_array_equal(g["pc_bar"][idx], o["Pc_bar"])


@pytest.mark.parametrize("n", [0, 1, 63, 64, 65, 129])
def test_edge_path_counts(n):
    r = M.mlmc_level(M.gbm(), 2, n, M.MLMC_FP32, M.MLMC_NESTED_CUBIC16, 1, 5)
    if n == 0:
        assert r["sum"][0] == 0 and r["sumsq"][1] == 0
        return
    o = mlmc.level_paths(2, np.arange(n), W.GBM, rv_mode=mlmc.RV_CUBIC, precision=fp.FP32, nested=True,
                         kahan=True, seed=5, stream=1)
    for k in range(3):
        assert sums_close(r["sum"][k], r["sumsq"][k], o, k), k


def test_path_offset_near_top_of_range():
    off, n = 2 ** 32 - 100, 100
    g = gpu_paths(W.GBM, 3, n, M.MLMC_FP64, 0, False, 0, 2, path_offset=off)
    o = mlmc.level_paths(3, np.arange(off, off + n), W.GBM, rv_mode=0, precision=fp.FP64, nested=False,
                         kahan=False, seed=2)
    assert np.all(close(g["pf_hat"], o["Pf_hat"], 1e-13))


def test_max_level_runs_and_matches():
    level, n = 16, 64
    g = gpu_paths(W.GBM, level, n, M.MLMC_FP32, M.MLMC_RV_PWL16, True, 1, 4)
    o = mlmc.level_paths(level, np.arange(n), W.GBM, rv_mode=mlmc.RV_PWL, precision=fp.FP32, nested=True,
                         kahan=True, seed=4, stream=1)
    assert np.all(close(g["pf_hat"], o["Pf_hat"], 1e-13))
    assert np.all(close(g["pc_hat"], o["Pc_hat"], 1e-13))
    assert np.all(close(g["pf_bar"], o["Pf_bar"], 1e-5))
    assert np.all(close(g["pc_bar"], o["Pc_bar"], 1e-5))


def test_deterministic_repeat():
    a = M.mlmc_level(M.gbm(payoff=1), 6, 100000, M.MLMC_FP32, M.MLMC_NESTED_PWL16, 0, 9)
    b = M.mlmc_level(M.gbm(payoff=1), 6, 100000, M.MLMC_FP32, M.MLMC_NESTED_PWL16, 0, 9)
    assert a["sum"][:3] == b["sum"][:3] and a["sumsq"][:3] == b["sumsq"][:3]


def test_invalid_arguments_rejected_on_gpu():
    with pytest.raises(M.MlmcError) as e:
        M.mlmc_level(M.gbm(), 3, 10, M.MLMC_FP32, M.MLMC_EXACT, 0, 0)
    assert e.value.code == M.MLMC_EINVAL
    with pytest.raises(M.MlmcError) as e:
        M.mlmc_level(M.gbm(T=-1.0), 3, 10, M.MLMC_FP32, M.MLMC_NESTED_PWL16, 0, 0)
    assert e.value.code == M.MLMC_EINVAL


def test_maximum_path_count_level0():
    """2^32 paths (the largest n_paths) at level 0: the sums are finite, the exact two-way mean
    is E[X_1] = 1 + mu within the central-limit bound, the four-way mean is 0 within its
    bound, and the two halves (path_offset 0 and 2^31) add up to the whole within rounding."""
    sde = M.gbm()
    whole = M.mlmc_level_run(M.level_args(sde, 0, 1 << 32, M.MLMC_FP32, M.MLMC_NESTED_PWL16, 0, 17))
    lo = M.mlmc_level_run(M.level_args(sde, 0, 1 << 31, M.MLMC_FP32, M.MLMC_NESTED_PWL16, 0, 17))
    hi = M.mlmc_level_run(M.level_args(sde, 0, 1 << 31, M.MLMC_FP32, M.MLMC_NESTED_PWL16, 0, 17,
                                       path_offset=1 << 31))
    m = float(1 << 32)
    assert all(math.isfinite(v) for v in whole["sum"][:3] + whole["sumsq"][:3])
    mean_e, var_e = E.level_stats(whole["sum"][2], whole["sumsq"][2], m)
    assert abs(mean_e - 1.05) < 5 * math.sqrt(var_e / m)
    assert abs(var_e / 0.04 - 1) < 1e-3
    mean_4, var_4 = E.level_stats(whole["sum"][1], whole["sumsq"][1], m)
    assert abs(mean_4) < 5 * math.sqrt(var_4 / m)
    for k in range(3):
        assert abs(lo["sum"][k] + hi["sum"][k] - whole["sum"][k]) <= 1e-12 * abs(whole["sumsq"][k]) ** 0.5 * m ** 0.5
        assert abs(lo["sumsq"][k] + hi["sumsq"][k] - whole["sumsq"][k]) <= 1e-12 * whole["sumsq"][k]


def test_full_size_sampled_paths_milstein_fp32():
    n, level = W.NESTED_FP32["n_paths"], 10
    sde = W.NESTED_FP32["sde"]
    g = gpu_paths(sde, level, n, M.MLMC_FP32, M.MLMC_RV_PWL16, True, 1, 0, scheme=M.MLMC_SCHEME_MILSTEIN)
    idx = W.sampled_paths(n, 48)
    o = mlmc.level_paths(level, idx, sde, rv_mode=mlmc.RV_PWL, precision=fp.FP32, nested=True, kahan=True,
                         seed=0, stream=1, scheme=mlmc.SCHEME_MILSTEIN)
    assert np.all(close(g["pf_hat"][idx], o["Pf_hat"], 1e-13))
    assert np.all(close(g["pc_hat"][idx], o["Pc_hat"], 1e-13))
    assert np.all(close(g["pf_bar"][idx], o["Pf_bar"], 1e-5))
    assert np.all(close(g["pc_bar"][idx], o["Pc_bar"], 1e-5))
