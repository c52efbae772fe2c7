"""Helpers for the GPU parity tests: device buffers and calls through the C-ABI binding."""

import numpy as np

import paper_2012_09739_amd as M


def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def gbm_struct(sde):
    return M.gbm(mu=sde["mu"], sigma=sde["sigma"], x0=sde["x0"], T=sde["T"], payoff=sde["payoff"],
                 strike=sde["strike"])


def rv_mode_code(rv, nested):
    if rv == 0:
        return M.MLMC_EXACT
    return rv + (4 if nested else 0)


def gpu_paths(sde, level, n_paths, precision, rv, nested, kahan, seed, *, diag=False, stream=None,
              path_offset=0, pset=0, scheme=0):
    """Per-path payoffs from mlmc_paths (same kernel and launch as the level sums)."""
    torch = torch_cuda()
    args = M.level_args(gbm_struct(sde), level, n_paths, precision, rv_mode_code(rv, nested), kahan, seed,
                        diag=int(diag), stream=stream, pset=pset, path_offset=path_offset, scheme=scheme)
    bufs = {k: torch.full((max(n_paths, 1),), float("nan"), dtype=torch.float64, device="cuda")
            for k in ("pf_hat", "pc_hat", "pf_bar", "pc_bar", "xf_tilde")}
    M.mlmc_paths(args, **bufs)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy()[:n_paths] for k, v in bufs.items()}


def gpu_uniforms(seed, stream, level, pset, path0, n_paths, n_steps):
    torch = torch_cuda()
    w = torch.zeros(n_paths * n_steps, dtype=torch.int32, device="cuda")
    M.mlmc_uniforms(seed, stream, level, pset, path0, n_paths, n_steps, w)
    torch.cuda.synchronize()
    return w.cpu().numpy().view(np.uint32).reshape(n_paths, n_steps)


def gpu_icdf(words, rv, precision):
    torch = torch_cuda()
    w = torch.from_numpy(np.asarray(words, dtype=np.uint32).view(np.int32)).cuda()
    out = torch.empty(w.numel(), dtype=torch.float64, device="cuda")
    M.mlmc_icdf(w, w.numel(), rv, precision, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()
