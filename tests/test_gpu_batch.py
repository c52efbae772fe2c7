"""GPU tests of the batched persistent sweep: every item equals the single-level call bit for
bit (same kernels' chunk partials, same fixed-order reduction), also when its chunks run
cooperatively on whole blocks, graph replays equal the eager launch, the oracle agrees on
small items, the autotuner keeps results unchanged, and the full 64-parameter-set x
15-level sweep runs."""

import math

import numpy as np
import pytest
import torch  # noqa: F401

import mlmc_workloads as W
from gpu_util import torch_cuda
from oracle import fp, mlmc
from test_gpu_parity import sums_close

import paper_2012_09739_amd as M

pytestmark = pytest.mark.gpu


def gbm_of(d):
    return M.gbm(mu=d["mu"], sigma=d["sigma"], x0=d["x0"], T=d["T"], payoff=d["payoff"], strike=d["strike"])


def make_items(psets, levels, paths_of, kahan16=1, kahan32=0, split=6, seed=0, payoff=0):
    items, meta = [], []
    for p, d in enumerate(psets):
        d = dict(d, payoff=payoff)
        for l in levels:
            prec = M.MLMC_FP16 if l <= split else M.MLMC_FP32
            k = kahan16 if prec == M.MLMC_FP16 else kahan32
            items.append(M.item(gbm_of(d), l, paths_of(l), prec, k, seed, pset=p, stream=1))
            meta.append((p, l, prec, k, d))
    return items, meta


def single_level(it, rv):
    torch = torch_cuda()
    args = M.level_args(it.sde, it.level, it.n_paths, it.precision, rv + 4, it.kahan, it.seed, stream=it.stream,
                        pset=it.pset)
    out = torch.zeros(8, dtype=torch.float64, device="cuda")
    M.mlmc_level_ex(args, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("rv", [M.MLMC_RV_PWL16, M.MLMC_RV_CUBIC16])
def test_batch_items_equal_single_level_calls(rv):
    torch = torch_cuda()
    psets = W.batch_parameter_sets(3, seed=5)
    items, meta = make_items(psets, range(9), lambda l: max(100, int(40000 / 2 ** l)) + 37 * l)
    out = torch.zeros((len(items), 8), dtype=torch.float64, device="cuda")
    plan = M.mlmc_batch_create(items, rv, out)
    try:
        M.mlmc_batch_run(plan)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        for i, it in enumerate(items):
            np.testing.assert_array_equal(got[i], single_level(it, rv), err_msg=str(meta[i][:4]))
    finally:
        M.mlmc_batch_destroy(plan)


@pytest.mark.parametrize("block_waves", [8, 4])
@pytest.mark.parametrize("kahan32", [0, 1])
@pytest.mark.parametrize("coop_level", [2, 7])
def test_cooperative_chunks_equal_single_level_calls(coop_level, kahan32, block_waves):
    # binary32 items from level 2 (one Philox call: a partial first phase) to 12 (1024 calls:
    # 342 phases of seven producers, 114 of three, the last one partial), path counts not
    # multiples of the chunk; blocks of eight and of four waves
    torch = torch_cuda()
    psets = W.batch_parameter_sets(2, seed=9)
    items, meta = make_items(psets, range(13), lambda l: max(70, 9000 >> l) + 5, split=1, kahan32=kahan32)
    out = torch.zeros((len(items), 8), dtype=torch.float64, device="cuda")
    cfg = M.mlmc_batch_cfg_t(16, 256, 25, coop_level, block_waves)
    plan = M.mlmc_batch_create(items, M.MLMC_RV_PWL16, out, cfg)
    try:
        M.mlmc_batch_run(plan)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        info, _ = M.mlmc_batch_info(plan)
        assert info.coop_level == coop_level and info.block_waves == block_waves
        for i, it in enumerate(items):
            np.testing.assert_array_equal(got[i], single_level(it, M.MLMC_RV_PWL16), err_msg=str(meta[i][:4]))
    finally:
        M.mlmc_batch_destroy(plan)


def test_graph_replays_equal_eager_with_work_between():
    torch = torch_cuda()
    psets = W.batch_parameter_sets(2, seed=1)
    items, _ = make_items(psets, range(8), lambda l: 5000 // (l + 1) + 1)
    out = torch.zeros((len(items), 8), dtype=torch.float64, device="cuda")
    plan = M.mlmc_batch_create(items, M.MLMC_RV_PWL16, out)
    try:
        M.mlmc_batch_run_eager(plan)
        torch.cuda.synchronize()
        eager = out.cpu().numpy().copy()
        for r in range(4):
            out.fill_(float("nan"))
            # unrelated eager work and synchronisations between the replays
            x = torch.randn(1 << 16, device="cuda").cumsum(0)
            single_level(items[r], M.MLMC_RV_PWL16)
            torch.cuda.synchronize()
            M.mlmc_batch_run(plan)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(out.cpu().numpy(), eager, err_msg="replay %d" % r)
            assert math.isfinite(float(x[-1]))
    finally:
        M.mlmc_batch_destroy(plan)


def test_batch_items_match_oracle():
    torch = torch_cuda()
    psets = W.batch_parameter_sets(2, seed=3)
    items, meta = make_items(psets, [0, 3, 6, 7, 9], lambda l: 300, payoff=1)
    out = torch.zeros((len(items), 8), dtype=torch.float64, device="cuda")
    plan = M.mlmc_batch_create(items, M.MLMC_RV_PWL16, out)
    try:
        M.mlmc_batch_run(plan)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
    finally:
        M.mlmc_batch_destroy(plan)
    for i, (p, l, prec, k, d) in enumerate(meta):
        o = mlmc.level_paths(l, np.arange(300), d, rv_mode=mlmc.RV_PWL, precision=prec, nested=True,
                             kahan=bool(k), seed=0, stream=1, pset=p)
        for t in range(3):
            assert sums_close(got[i][t], got[i][4 + t], o, t), (p, l, t)


def test_autotune_keeps_results_and_returns_valid_shape(tmp_path, monkeypatch):
    torch = torch_cuda()
    monkeypatch.setenv("MLMC_AUTOTUNE_CACHE", str(tmp_path / "tune.txt"))
    psets = W.batch_parameter_sets(2, seed=2)
    items, _ = make_items(psets, range(10), lambda l: max(256, 20000 >> l))
    out = torch.zeros((len(items), 8), dtype=torch.float64, device="cuda")
    plan = M.mlmc_batch_create(items, M.MLMC_RV_PWL16, out)
    try:
        M.mlmc_batch_run(plan)
        torch.cuda.synchronize()
        before = out.cpu().numpy().copy()
        best = M.mlmc_batch_autotune(plan, 1)
        assert 4 <= best.waves_per_cu <= 32 and best.task_steps >= 1
        cfg, n_tasks = M.mlmc_batch_info(plan)
        assert (cfg.waves_per_cu, cfg.task_steps, cfg.priority_level, cfg.coop_level, cfg.block_waves) == (
            best.waves_per_cu, best.task_steps, best.priority_level, best.coop_level, best.block_waves)
        assert best.block_waves in (4, 8) and best.waves_per_cu % best.block_waves == 0
        assert n_tasks > 0
        out.zero_()
        M.mlmc_batch_run(plan)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy(), before)
        assert (tmp_path / "tune.txt").exists()
    finally:
        M.mlmc_batch_destroy(plan)
    # a new plan for the same items picks the cached shape
    plan2 = M.mlmc_batch_create(items, M.MLMC_RV_PWL16, out)
    try:
        cfg2, _ = M.mlmc_batch_info(plan2)
        assert (cfg2.waves_per_cu, cfg2.task_steps, cfg2.priority_level, cfg2.coop_level, cfg2.block_waves) == (
            best.waves_per_cu, best.task_steps, best.priority_level, best.coop_level, best.block_waves)
    finally:
        M.mlmc_batch_destroy(plan2)


def test_full_ragged_sweep_64_psets_15_levels():
    torch = torch_cuda()
    psets = W.batch_parameter_sets(W.BATCH_PSETS, seed=0)
    items, meta = make_items(psets, W.BATCH_LEVELS, W.batch_paths)
    assert len(items) == 960
    out = torch.zeros((len(items), 8), dtype=torch.float64, device="cuda")
    plan = M.mlmc_batch_create(items, M.MLMC_RV_PWL16, out)
    try:
        M.mlmc_batch_run(plan)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
    finally:
        M.mlmc_batch_destroy(plan)
    assert np.all(np.isfinite(got))
    for i in (0, 6, 7, 14, 15 * 63 + 0, 15 * 63 + 14):
        np.testing.assert_array_equal(got[i], single_level(items[i], M.MLMC_RV_PWL16), err_msg=str(meta[i][:4]))


def test_invalid_items_rejected():
    torch = torch_cuda()
    out = torch.zeros((1, 8), dtype=torch.float64, device="cuda")
    bad = M.item(M.gbm(), 3, 100, M.MLMC_FP64, 0)
    with pytest.raises(M.MlmcError) as e:
        M.mlmc_batch_create([bad], M.MLMC_RV_PWL16, out)
    assert e.value.code == M.MLMC_EINVAL


def test_item_times_account_for_the_sweep():
    """Per-item wavefront time (cost attribution, Section 3's c_l per item): positive, not
    accumulated across replays, bounded by resident waves x elapsed time, and proportional
    to the work within one arithmetic variant."""
    torch = torch_cuda()
    psets = W.batch_parameter_sets(8, seed=4)
    items, meta = make_items(psets, W.BATCH_LEVELS, W.batch_paths)
    out = torch.zeros((len(items), 8), dtype=torch.float64, device="cuda")
    plan = M.mlmc_batch_create(items, M.MLMC_RV_PWL16, out)
    try:
        cfg, _ = M.mlmc_batch_info(plan)
        waves = cfg.waves_per_cu * torch.cuda.get_device_properties(0).multi_processor_count
        totals = []
        for _ in range(2):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            M.mlmc_batch_run(plan)
            e1.record()
            torch.cuda.synchronize()
            t = np.array(M.mlmc_batch_item_times(plan, len(items)))
            elapsed = e0.elapsed_time(e1) * 1e-3
            assert np.all(t > 0)
            assert t.sum() <= waves * elapsed * 1.05, (t.sum(), waves, elapsed)
            totals.append(t.sum())
    finally:
        M.mlmc_batch_destroy(plan)
    assert 0.5 < totals[1] / totals[0] < 2.0   # reset on every replay, not accumulated
    steps = np.array([it.n_paths << it.level for it in items], dtype=np.float64)
    per = t / steps
    fp32 = np.array([m[1] >= 9 for m in meta])   # binary32 items with whole 64-path chunks busy
    ratio = per[fp32].max() / per[fp32].min()
    assert ratio < 4.0, ratio
