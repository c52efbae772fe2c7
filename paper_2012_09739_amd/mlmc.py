"""Python binding of libmlmc (ctypes): argument marshalling only.

Every entry point has the name and meaning of its C counterpart in include/mlmc.h; all
computation happens in the HIP library.  Device buffers are passed as PyTorch CUDA
(HIP) tensors or raw integer addresses; the stream defaults to PyTorch's current stream.
The library must have been built (paper_2012_09739_amd.build); there is no fallback.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# MLMC_LIBRARY selects another build of the same library (the host-sanitizer build of the
# CPU tests); by default the in-tree libmlmc.so
LIB_PATH = os.environ.get("MLMC_LIBRARY") or os.path.join(HERE, "libmlmc.so")

MLMC_OK, MLMC_EINVAL, MLMC_ENOMEM, MLMC_ENODEV, MLMC_EHIP, MLMC_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
MLMC_FP64, MLMC_FP32, MLMC_FP16 = 0, 1, 2
MLMC_BF16 = 3   # emulated bfloat16 (dyadic approximations only)
MLMC_RV_EXACT, MLMC_RV_PWL16, MLMC_RV_CUBIC16, MLMC_RV_MLP, MLMC_RV_PCONST4096 = 0, 1, 2, 3, 4
MLMC_EXACT, MLMC_APPROX_PWL16, MLMC_APPROX_CUBIC16, MLMC_APPROX_MLP = 0, 1, 2, 3
MLMC_NESTED_PWL16, MLMC_NESTED_CUBIC16, MLMC_NESTED_MLP = 5, 6, 7
MLMC_APPROX_PCONST4096, MLMC_NESTED_PCONST4096 = 4, 8
MLMC_TERM_TWO_WAY, MLMC_TERM_FOUR_WAY, MLMC_TERM_TWO_WAY_EXACT, MLMC_TERM_ROUNDING = 0, 1, 2, 3
MLMC_PAYOFF_X, MLMC_PAYOFF_CALL = 0, 1
MLMC_SCHEME_EM, MLMC_SCHEME_MILSTEIN = 0, 1

ERROR_NAMES = {MLMC_EINVAL: "MLMC_EINVAL", MLMC_ENOMEM: "MLMC_ENOMEM", MLMC_ENODEV: "MLMC_ENODEV",
               MLMC_EHIP: "MLMC_EHIP", MLMC_EUNSUPPORTED: "MLMC_EUNSUPPORTED"}


class MlmcError(RuntimeError):
    def __init__(self, code, message):
        super().__init__("%s (%d): %s" % (ERROR_NAMES.get(code, "?"), code, message))
        self.code = code


class mlmc_gbm_t(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_double), ("sigma", ctypes.c_double), ("x0", ctypes.c_double),
                ("T", ctypes.c_double), ("payoff", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("strike", ctypes.c_double)]


class mlmc_result_t(ctypes.Structure):
    _fields_ = [("sum", ctypes.c_double * 4), ("sumsq", ctypes.c_double * 4), ("n_paths", ctypes.c_uint64),
                ("path_steps", ctypes.c_uint64), ("cost_seconds", ctypes.c_double)]


class mlmc_level_args_t(ctypes.Structure):
    _fields_ = [("sde", mlmc_gbm_t), ("level", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("rv_mode", ctypes.c_int32), ("kahan", ctypes.c_int32), ("diag", ctypes.c_int32),
                ("stream", ctypes.c_uint32), ("pset", ctypes.c_uint32), ("scheme", ctypes.c_uint32),
                ("seed", ctypes.c_uint64), ("n_paths", ctypes.c_uint64), ("path_offset", ctypes.c_uint64)]


class mlmc_item_t(ctypes.Structure):
    _fields_ = [("sde", mlmc_gbm_t), ("level", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("kahan", ctypes.c_int32), ("pset", ctypes.c_uint32), ("stream", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("n_paths", ctypes.c_uint64), ("seed", ctypes.c_uint64)]


class mlmc_batch_cfg_t(ctypes.Structure):
    _fields_ = [("waves_per_cu", ctypes.c_int32), ("task_steps", ctypes.c_int32),
                ("priority_level", ctypes.c_int32), ("coop_level", ctypes.c_int32),
                ("block_waves", ctypes.c_int32)]


class mlmc_mlp_cfg_t(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("n_pairs", ctypes.c_uint32), ("batch", ctypes.c_uint32),
                ("epochs", ctypes.c_uint32), ("lr", ctypes.c_float), ("lr_final", ctypes.c_float),
                ("reserved", ctypes.c_uint32)]


_P = ctypes.c_void_p
_SIGNATURES = {
    "mlmc_init": (ctypes.c_int, [ctypes.c_int]),
    "mlmc_shutdown": (ctypes.c_int, []),
    "mlmc_level": (ctypes.c_int, [ctypes.POINTER(mlmc_gbm_t), ctypes.c_int, ctypes.c_uint64, ctypes.c_int,
                                  ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.POINTER(mlmc_result_t)]),
    "mlmc_level_run": (ctypes.c_int, [ctypes.POINTER(mlmc_level_args_t), ctypes.POINTER(mlmc_result_t)]),
    "mlmc_level_set_run": (ctypes.c_int, [ctypes.POINTER(mlmc_level_args_t), ctypes.c_int,
                                          ctypes.POINTER(mlmc_result_t), ctypes.POINTER(ctypes.c_double)]),
    "mlmc_level_ex": (ctypes.c_int, [ctypes.POINTER(mlmc_level_args_t), _P, _P, ctypes.c_size_t, _P]),
    "mlmc_level_noalloc": (ctypes.c_int, [ctypes.POINTER(mlmc_level_args_t), _P, _P]),
    "mlmc_level_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(mlmc_level_args_t)]),
    "mlmc_paths": (ctypes.c_int, [ctypes.POINTER(mlmc_level_args_t), _P, _P, _P, _P, _P, _P]),
    "mlmc_uniforms": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_uint32,
                                     ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, _P, _P]),
    "mlmc_icdf": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.c_int, ctypes.c_int, _P, _P]),
    "mlmc_table": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]),
    "mlmc_pconst_table": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_double)]),
    "mlmc_last_error": (ctypes.c_char_p, []),
    "mlmc_batch_create": (ctypes.c_int, [ctypes.POINTER(mlmc_item_t), ctypes.c_int, ctypes.c_int,
                                         ctypes.POINTER(mlmc_batch_cfg_t), _P, ctypes.POINTER(_P)]),
    "mlmc_batch_run": (ctypes.c_int, [_P, _P]),
    "mlmc_batch_run_eager": (ctypes.c_int, [_P, _P]),
    "mlmc_batch_autotune": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(mlmc_batch_cfg_t)]),
    "mlmc_batch_info": (ctypes.c_int, [_P, ctypes.POINTER(mlmc_batch_cfg_t), ctypes.POINTER(ctypes.c_uint64)]),
    "mlmc_batch_item_times": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double), _P]),
    "mlmc_batch_destroy": (ctypes.c_int, [_P]),
    "mlmc_mlp_pairs": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, _P, _P, _P, _P]),
    "mlmc_mlp_grad": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, _P, _P, _P]),
    "mlmc_mlp_train": (ctypes.c_int, [ctypes.POINTER(mlmc_mlp_cfg_t), _P, _P, _P]),
    "mlmc_mlp_load": (ctypes.c_int, [_P, _P]),
}

_lib = None


def lib():
    """The loaded libmlmc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmlmc.so is not built: run `python -m paper_2012_09739_amd.build` "
                               "(there is no CPU fallback)")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def exported_symbols():
    return list(_SIGNATURES)


def _check(rc):
    if rc != MLMC_OK:
        raise MlmcError(rc, lib().mlmc_last_error().decode())


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(s):
    if s is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(s, int):
        return s
    return s.cuda_stream


def gbm(mu=0.05, sigma=0.2, x0=1.0, T=1.0, payoff=MLMC_PAYOFF_X, strike=1.0):
    """A GBM problem dX = mu X dt + sigma X dW (defaults: the paper's test problem)."""
    return mlmc_gbm_t(mu, sigma, x0, T, payoff, 0, strike)


def level_args(sde, level, n_paths, precision, rv_mode, kahan=0, seed=0, *, diag=0, stream=None, pset=0,
               path_offset=0, scheme=MLMC_SCHEME_EM):
    """mlmc_level_args_t; stream defaults to 1 for nested modes and 0 otherwise."""
    if stream is None:
        stream = 1 if rv_mode >= MLMC_NESTED_PWL16 else 0
    return mlmc_level_args_t(sde, level, precision, rv_mode, int(kahan), int(diag), stream, pset, scheme, seed,
                             n_paths, path_offset)


def _result_dict(r):
    return {"sum": list(r.sum), "sumsq": list(r.sumsq), "n_paths": r.n_paths, "path_steps": r.path_steps,
            "cost_seconds": r.cost_seconds}


def mlmc_init(device=0):
    _check(lib().mlmc_init(device))


def mlmc_shutdown():
    _check(lib().mlmc_shutdown())


def mlmc_level(sde, level, n_paths, precision, rv_mode, kahan, seed):
    """Synchronous level call; returns dict(sum, sumsq, n_paths, path_steps, cost_seconds)."""
    out = mlmc_result_t()
    _check(lib().mlmc_level(ctypes.byref(sde), level, n_paths, precision, rv_mode, int(kahan), seed,
                            ctypes.byref(out)))
    return _result_dict(out)


def mlmc_level_run(args):
    """Synchronous level call with the full argument set; returns the same dict as mlmc_level."""
    out = mlmc_result_t()
    _check(lib().mlmc_level_run(ctypes.byref(args), ctypes.byref(out)))
    return _result_dict(out)


def mlmc_level_set_run(args_list):
    """Level calls issued together over the library's streams; returns (list of result dicts
    as mlmc_level_run, device seconds from the first start to the last end)."""
    n = len(args_list)
    arr = (mlmc_level_args_t * n)(*args_list)
    res = (mlmc_result_t * n)()
    span = ctypes.c_double(0.0)
    _check(lib().mlmc_level_set_run(arr, n, res, ctypes.byref(span)))
    return [_result_dict(r) for r in res], span.value


def mlmc_level_workspace_bytes(args):
    return int(lib().mlmc_level_workspace_bytes(ctypes.byref(args)))


def mlmc_level_ex(args, d_out, workspace=None, workspace_bytes=0, stream=None):
    """Asynchronous level call writing 8 doubles (sums, sums of squares) to d_out."""
    if workspace is not None and not workspace_bytes:
        workspace_bytes = workspace.numel() * workspace.element_size()
    _check(lib().mlmc_level_ex(ctypes.byref(args), _ptr(d_out), _ptr(workspace), workspace_bytes,
                               _stream(stream)))


def mlmc_level_noalloc(args, d_out, stream=None):
    """mlmc_level_ex with the library's fixed device scratch (allocates nothing; needs mlmc_init)."""
    _check(lib().mlmc_level_noalloc(ctypes.byref(args), _ptr(d_out), _stream(stream)))


def mlmc_paths(args, pf_hat=None, pc_hat=None, pf_bar=None, pc_bar=None, xf_tilde=None, stream=None):
    _check(lib().mlmc_paths(ctypes.byref(args), _ptr(pf_hat), _ptr(pc_hat), _ptr(pf_bar), _ptr(pc_bar),
                            _ptr(xf_tilde), _stream(stream)))


def mlmc_uniforms(seed, stream_id, level, pset, path0, n_paths, n_steps, d_words, stream=None):
    _check(lib().mlmc_uniforms(seed, stream_id, level, pset, path0, n_paths, n_steps, _ptr(d_words),
                               _stream(stream)))


def mlmc_icdf(d_words, n, rv, precision, d_out, stream=None):
    _check(lib().mlmc_icdf(_ptr(d_words), n, rv, precision, _ptr(d_out), _stream(stream)))


def mlmc_table(rv, precision):
    """16 x 4 list of coefficients (rounded to precision, widened to binary64)."""
    buf = (ctypes.c_double * 64)()
    _check(lib().mlmc_table(rv, precision, buf))
    return [[buf[4 * j + i] for i in range(4)] for j in range(16)]


def mlmc_pconst_table(precision):
    """The 2048 lower-half cell means of MLMC_RV_PCONST4096 (rounded to precision, widened)."""
    buf = (ctypes.c_double * 2048)()
    _check(lib().mlmc_pconst_table(precision, buf))
    return list(buf)


def item(sde, level, n_paths, precision, kahan=0, seed=0, *, pset=0, stream=1):
    """One (parameter set, level) item of a batched sweep (nested samples)."""
    return mlmc_item_t(sde, level, precision, int(kahan), pset, stream, 0, n_paths, seed)


def mlmc_batch_create(items, rv, d_out, cfg=None):
    """Plan for a list of mlmc_item_t; d_out: device tensor of len(items) x 8 doubles.
    Returns an opaque plan handle (int)."""
    arr = (mlmc_item_t * len(items))(*items)
    plan = ctypes.c_void_p()
    _check(lib().mlmc_batch_create(arr, len(items), rv, ctypes.byref(cfg) if cfg is not None else None,
                                   _ptr(d_out), ctypes.byref(plan)))
    return plan.value


def mlmc_batch_run(plan, stream=None):
    _check(lib().mlmc_batch_run(plan, _stream(stream)))


def mlmc_batch_run_eager(plan, stream=None):
    _check(lib().mlmc_batch_run_eager(plan, _stream(stream)))


def mlmc_batch_autotune(plan, repeats=3):
    best = mlmc_batch_cfg_t()
    _check(lib().mlmc_batch_autotune(plan, repeats, ctypes.byref(best)))
    return best


def mlmc_batch_info(plan):
    cfg = mlmc_batch_cfg_t()
    n = ctypes.c_uint64()
    _check(lib().mlmc_batch_info(plan, ctypes.byref(cfg), ctypes.byref(n)))
    return cfg, n.value


def mlmc_batch_item_times(plan, n_items, stream=None):
    """Wavefront-seconds spent on each of the plan's n_items items in its last run."""
    buf = (ctypes.c_double * n_items)()
    _check(lib().mlmc_batch_item_times(plan, buf, _stream(stream)))
    return list(buf)


def mlmc_batch_destroy(plan):
    _check(lib().mlmc_batch_destroy(plan))


def mlp_cfg(seed=0, n_pairs=2 ** 20, batch=4096, epochs=40, lr=1e-2, lr_final=1e-5):
    return mlmc_mlp_cfg_t(seed, n_pairs, batch, epochs, lr, lr_final, 0)


def mlmc_mlp_pairs(seed, first, n, d_x, d_target, d_words=None, stream=None):
    _check(lib().mlmc_mlp_pairs(seed, first, n, _ptr(d_words), _ptr(d_x), _ptr(d_target), _stream(stream)))


def mlmc_mlp_grad(d_params, seed, first, n, d_grad, d_loss=None, stream=None):
    _check(lib().mlmc_mlp_grad(_ptr(d_params), seed, first, n, _ptr(d_grad), _ptr(d_loss), _stream(stream)))


def mlmc_mlp_train(cfg, d_params, stream=None):
    """Trains in place (device tensor of 321 floats); returns the per-epoch losses."""
    hist = (ctypes.c_float * cfg.epochs)()
    _check(lib().mlmc_mlp_train(ctypes.byref(cfg), _ptr(d_params), hist, _stream(stream)))
    return list(hist)


def mlmc_mlp_load(d_params, stream=None):
    _check(lib().mlmc_mlp_load(_ptr(d_params), _stream(stream)))


def mlmc_last_error():
    return lib().mlmc_last_error().decode()

