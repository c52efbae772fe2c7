"""Level calls captured in a graph: mlmc_level_ex with a caller workspace on a capturing
stream records only kernel launches (no allocation, no memset node), so a captured sequence
of levels replays to the same bits as the eager calls, replay after replay, with unrelated
eager work and synchronisations in between."""

import math

import numpy as np
import pytest

import paper_2012_09739_amd as M

pytestmark = pytest.mark.gpu


def test_captured_level_sequence_replays_equal_eager():
    import torch
    call = M.gbm(payoff=M.MLMC_PAYOFF_CALL)
    args = [M.level_args(call, l, 50000 + 17 * l, M.MLMC_FP32, M.MLMC_NESTED_PWL16, l % 2, 3) for l in (0, 3, 7)]
    args.append(M.level_args(call, 5, 30000, M.MLMC_FP16, M.MLMC_NESTED_CUBIC16, 1, 3, diag=1))
    args.append(M.level_args(call, 4, 20000, M.MLMC_FP64, M.MLMC_EXACT, 0, 3, scheme=M.MLMC_SCHEME_MILSTEIN))
    # deep calls with few chunks: one block per chunk (nested binary32, plain binary64)
    args.append(M.level_args(call, 10, 1000, M.MLMC_FP32, M.MLMC_NESTED_PWL16, 1, 3))
    args.append(M.level_args(call, 9, 777, M.MLMC_FP64, M.MLMC_EXACT, 0, 3))
    out = torch.zeros((len(args), 8), dtype=torch.float64, device="cuda")
    ws = [torch.empty(M.mlmc_level_workspace_bytes(a) // 8 + 1, dtype=torch.float64, device="cuda") for a in args]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for a, o, w in zip(args, out, ws):
            M.mlmc_level_ex(a, o, w, stream=s)
    torch.cuda.synchronize()
    eager = out.cpu().numpy().copy()
    assert np.all(np.isfinite(eager[:, :3]))
    assert np.all(np.isfinite(eager[-1, [0, 4]]))

    g = torch.cuda.CUDAGraph()
    out.fill_(float("nan"))
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        for a, o, w in zip(args, out, ws):
            M.mlmc_level_ex(a, o, w, stream=s)
    for r in range(4):
        out.fill_(float("nan"))
        x = torch.randn(1 << 16, device="cuda").cumsum(0)   # unrelated eager work
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy(), eager, err_msg="replay %d" % r)
        assert math.isfinite(float(x[-1]))
