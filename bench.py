"""Benchmark: nested four-way MLMC in binary32 on one MI355X.

Workload (one "step" = one pass of the whole hot path over one batch of synthetic input):
geometric Brownian motion mu = 0.05, sigma = 0.2, X0 = 1, T = 1, European call
max(X_T - 1, 0); nested four-way samples (exact binary64 pair and approximate binary32
pair from the same Philox4x32-10 uniforms, piecewise-linear inverse CDF on 16 dyadic
intervals) at levels 0..10 with 2^20 paths per level, once without and once with Kahan
compensation.  Each sample yields the four-way difference and both two-way differences
with on-device binary64 sums and sums of squares.

Metric: coupled path-steps per second (one coupled path-step = one fine time step of one
coupled sample, including its share of the coarse step) -- inputs are seeds, resident on
the device by construction.  A step is one pass of the 22 level calls, captured once as a
hipGraph and replayed (every replay's sums are checked equal to the eager pass's).  Besides the headline number the JSON line reports the plain
binary64 estimator's throughput at the same sizes and the speed-up of the nested
binary32 estimator over it at equal total MLMC variance (T^ / T-, from measured
per-level variances and device costs), the roofline of the dominant kernel and the CPU
oracle timed on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

LEVELS = list(range(11))
N_PATHS = 2 ** 20
SEED = 0
# VALU issue peak of MI355X in slots: a slot is one wavefront instruction at the binary64
# FMA rate, 64 lane-operations per CU per clock, so the peak is 256 CUs x 64 x 2.4 GHz
# = 39.32 T lane-slots/s (the binary64 vector peak 78.6 TFLOP/s / 2 flops per FMA).  The
# issue cost of an opcode in slots is measured by the issue-rate probes (libvalurates.so,
# report leg "valu_rates"; profiles/valu_issue_rates_gfx950.md): 1/2 for binary32 and
# scalar binary16 add / mul / fma, 32-bit add / sub / and / xor / shifts, the three-input
# xor and v_cndmask; 1 for binary64 arithmetic, packed binary16, the 32x32->64 products,
# conversions, clz, min, lshl_or, perm, med3, compares, clamped v_max_f32 and 64-bit
# shifts and moves; 2 for scalar binary16 fma, mixed-precision fma, 16-bit bitop3 and the
# transcendental unit (exp, log, sqrt, rcp).
PEAK_VALU_TOPS = 256 * 64 * 2.4e9 / 1e12
# vector peaks of MI355X (TFLOP/s): binary64 and binary32 published; packed binary16 at the
# rate the probes measure for v_pk_fma_f16 (one instruction per slot, two FMAs per lane)
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "f16": 157.3}
# The dominant kernels, each timed alone: HIP events on the launching stream around
# mlmc_paths with no per-path outputs, which launches exactly the level kernel of
# mlmc_level_ex (same instance and grid) without the two kernels of the chunk reduction.
# Per coupled path-step, counted in the AMD assembly of the kernels' step loop (one trip =
# one Philox call: four fine steps of a lane's path, two packed paths in binary16; the
# branch of the deep cells of the exact variable, taken with probability 2^-11, excluded):
#   slots  weighted issue cost of the loop's VALU instructions (the weights above)
#   valu   VALU instructions; rocprofv3's SQ_INSTS_VALU per launch agrees within 2% (the
#          rest is the rows' set-up and reduction)
#   flops  floating-point operations by precision (an FMA counts 2, a packed binary16
#          operation 2 or 4)
ROOFLINE_KERNELS = {
    "fp32": dict(precision="MLMC_FP32", mode="MLMC_NESTED_PWL16", kahan=1, level=10, n_paths=2 ** 20,
                 slots=38.25, valu=52.25, flops={"f64": 24.5, "f32": 14.5},
                 kernel="level_kernel<FP32, PWL16, nested, Kahan> at level 10 (2^20 paths x 1024 steps)"),
    "fp16": dict(precision="MLMC_FP16", mode="MLMC_NESTED_CUBIC16", kahan=1, level=6, n_paths=2 ** 24,
                 slots=41.75, valu=52.0, flops={"f64": 24.5, "f32": 1.0, "f16": 18.5},
                 kernel="level_kernel<FP16, CUBIC16, nested, Kahan> at level 6 (2^24 paths x 64 steps)"),
}
# the sources and build flags the counts above were taken from (sha256 of ISA_SOURCES)
ISA_SOURCES_SHA256 = "66e051ae0572e5bdafd00bc7e2e43ce7b6c4ecbbbcdfb3137aa73c03fe74e7c7"
# HBM bytes per launch of each kernel from rocprofv3 FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 (KiB;
# scale factors from a 256 MiB device copy), valid for the kernel sources hashed below
TRAFFIC_BYTES_PER_LAUNCH = {"fp32": (218.438 * 2.0 + 1024.0) * 1024, "fp16": (243.938 * 2.0 + 8192.0) * 1024}
TRAFFIC_SOURCES_SHA256 = "9db52fa51560ac6e26823a97d2be99711adc8cba1834fd23d181707384d88fe8"
# what a kernel's instructions depend on: its sources and the build flags
ISA_SOURCES = ("csrc/level_kernel.h", "csrc/level_launch.h", "csrc/icdf.h", "csrc/philox.h", "csrc/mlp.h",
               "csrc/internal.h", "csrc/level_f32.hip", "csrc/level_f16.hip", "csrc/icdf_exact_coeffs.h", "build.py")
# and its memory traffic besides: the launch grid (the number of partial rows)
KERNEL_SOURCES = ISA_SOURCES + ("csrc/abi.cpp",)


def sources_sha256(names):
    import hashlib
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, "paper_2012_09739_amd", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def kernel_sources_sha256():
    return sources_sha256(KERNEL_SOURCES)


def traffic_bytes(key):
    """The counter-derived traffic if the kernel sources are unchanged since it was taken."""
    if TRAFFIC_BYTES_PER_LAUNCH.get(key) is None or kernel_sources_sha256() != TRAFFIC_SOURCES_SHA256:
        return None
    return TRAFFIC_BYTES_PER_LAUNCH[key]


REPORT_LEGS = ("plain", "fp16", "batch", "mlp", "sweep", "adaptive", "milstein", "pconst", "marginal", "valu_rates")
# opcodes of the issue-rate probes (include/valu_rates.h order)
VALU_OPS = ("v_fma_f64", "v_mul_f64", "v_add_f64", "v_fma_f32", "v_mul_f32", "v_pk_fma_f16", "v_pk_mul_f16",
            "v_fma_f16", "v_bitop3_b32 (xor3)", "v_add_u32", "v_mul_lo_u32", "v_mul_hi_u32", "v_ffbh_u32",
            "v_exp_f32", "v_rcp_f32", "v_med3_f32", "v_mad_u64_u32", "v_cvt_f32_f64 + v_cvt_f64_f32",
            "v_cvt_f16_f32 + v_cvt_f32_f16", "v_min_u32", "v_lshl_or_b32", "v_cmp_gt_u32 + v_cndmask_b32",
            "v_perm_b32", "v_and_b32", "v_ashrrev_i32", "v_add_f16", "v_mul_f16", "v_pk_add_f16", "v_cvt_pk_f16_f32",
            "v_cvt_f32_u32", "v_cvt_f64_u32", "v_lshlrev_b64", "v_lshl_add_u64", "v_mov_b64",
            "v_max_f32 clamp", "v_sub_u32 clamp", "v_lshrrev_b32", "v_fma_mixlo_f16", "v_bitop3_b16", "v_log_f32",
            "v_sqrt_f32", "v_cmp_gt_u32")


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-speedup", action="store_true", help="skip the equal-variance legs")
    p.add_argument("--no-reports", action="store_true",
                   help="skip the report legs of the other workloads (fp64 plain, fp16, batch, mlp, ...)")
    p.add_argument("--reports", default=",".join(REPORT_LEGS),
                   help="comma-separated report legs to run: " + ", ".join(REPORT_LEGS))
    p.add_argument("--calibrate-copy", action="store_true",
                   help="also run a device copy of known size (HBM counter calibration)")
    p.add_argument("--profile", choices=("roofline", "valu_rates", "coop"),
                   help="profiling run: only the dominant kernels' timed launches (roofline), only "
                        "the issue-rate probes, or only deep single-level calls with few chunks "
                        "(cooperative kernel), printed as one JSON line without the headline metric")
    return p.parse_args()


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: it measures the single-GPU kernel; "
              "paths shard across GPUs by path_offset but no multi-GPU run is made",
              file=sys.stderr)
        sys.exit(2)
    if a.profile:
        profile_run(a.profile, a.calibrate_copy)
        return
    # the CPU oracle runs first, in worker processes started before anything touches the GPU
    cpu = None if a.no_cpu_baseline else cpu_baseline()

    import torch

    import paper_2012_09739_amd as M
    from paper_2012_09739_amd import estimators as E

    torch.cuda.set_device(0)
    M.mlmc_init(0)
    stream = torch.cuda.current_stream()
    call = M.gbm(payoff=M.MLMC_PAYOFF_CALL)
    args = {k: [M.level_args(call, l, N_PATHS, M.MLMC_FP32, M.MLMC_NESTED_PWL16, k, SEED) for l in LEVELS]
            for k in (0, 1)}
    out = torch.zeros((2, len(LEVELS), 8), dtype=torch.float64, device="cuda")
    ws_bytes = max(M.mlmc_level_workspace_bytes(x) for x in args[0])
    # the 22 independent level calls, deepest first, alternate between two streams (default
    # priority), each stream with its own workspace, as mlmc_level_set_run issues a level set:
    # one call's short coarse kernels and launch gaps overlap the other stream's work
    side = [torch.cuda.Stream() for _ in range(2)]
    ws = [torch.empty(ws_bytes // 8 + 1, dtype=torch.float64, device="cuda") for _ in side]
    order = sorted(((i, l, k) for k in (0, 1) for i, l in enumerate(LEVELS)), key=lambda c: -c[1])
    top = LEVELS[-1]

    def step(st):
        for s in side:
            s.wait_stream(st)
        for j, (i, l, k) in enumerate(order):
            M.mlmc_level_ex(args[k][i], out[k, i], ws[j % 2], ws_bytes, side[j % 2])
        for s in side:
            st.wait_stream(s)

    # one pass (22 level calls, each its level kernel and its reduction) captured once as a
    # hipGraph and replayed: the GPU work of a step without per-launch host overhead
    for _ in range(max(1, a.warmup)):
        step(stream)
    torch.cuda.synchronize()
    eager = out.cpu().numpy().copy()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step(torch.cuda.current_stream())
    torch.cuda.synchronize()
    for _ in range(a.warmup):
        graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        graph.replay()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    steps_per_pass = 2 * N_PATHS * sum(2 ** l for l in LEVELS)
    seconds = t1 - t0
    value = a.steps * steps_per_pass / seconds
    sums = out.cpu().numpy()
    assert all(math.isfinite(v) for v in sums.ravel()), "non-finite level sums"
    # every replay computes the same samples as the eager pass, bit for bit
    assert (sums == eager).all(), "graph replay differs from the eager pass"
    # the dominant call alone, eagerly: level 10 with Kahan updates, kernel plus reduction
    ev = []
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        M.mlmc_level_ex(args[1][top], out[1, top], ws[0], ws_bytes, stream)
        e1.record(stream)
        ev.append((e0, e1))
    torch.cuda.synchronize()
    launch_ms = sum(e0.elapsed_time(e1) for e0, e1 in ev) / len(ev)

    roof = {k: roofline_block(M, torch, k) for k in ROOFLINE_KERNELS}
    roof["fp32"]["call_ms_with_reduction"] = launch_ms

    extra = {}
    if not a.no_speedup:
        extra = equal_variance_report(M, E, call)

    if a.calibrate_copy:
        src = torch.empty(256 * 2 ** 20 // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        extra["copy_calibration_bytes"] = 2 * src.numel() * 4

    if not a.no_reports:
        legs = tuple(x for x in a.reports.split(",") if x)
        unknown = [x for x in legs if x not in REPORT_LEGS]
        if unknown:
            print("unknown report legs: %s" % ", ".join(unknown), file=sys.stderr)
            sys.exit(2)
        extra["reports"] = reports(M, E, torch, legs)

    line = {
        "metric": "coupled path-steps/s FP16/FP32 vs FP64 at equal MLMC variance; % VALU peak",
        "value": value,
        "unit": "coupled path-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": seconds / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic (seeded Philox4x32-10 uniforms; no dataset)",
        "config": {"workload": "nested four-way MLMC, GBM mu=0.05 sigma=0.2 X0=1 T=1, call K=1, "
                               "binary32 approximate pair with piecewise-linear inverse CDF on 16 dyadic "
                               "intervals, binary64 exact pair, levels 0..10, 2^20 paths/level, "
                               "Kahan off and on; one pass of the 22 level calls (deepest first, over two "
                               "streams) replayed as a hipGraph",
                   "levels": LEVELS, "paths_per_level": N_PATHS, "kahan": [0, 1],
                   "coupled_path_steps_per_step": steps_per_pass, "parallelism": "single GPU"},
        "roofline": roof["fp32"],
        "roofline_fp16": roof["fp16"],
        "cpu_baseline": cpu,
    }
    line["speedup_equal_variance"] = equal_variance_summary(extra)
    line.update(extra)
    print(json.dumps(line), flush=True)


def equal_variance_summary(extra):
    """T^ / T- (plain binary64 time over nested time at equal total MLMC variance, Section 3)
    of every configuration the run measured, gathered at the top level of the line."""
    out = {}
    ev = extra.get("equal_variance", {})
    for tag, key in (("fp32_pwl16_levels0to10", "fp32"), ("fp32_pwl16_kahan_levels0to10", "fp32_kahan")):
        if key in ev:
            out[tag] = ev[key]["speedup_T_hat_over_T_bar"]
            out[tag + "_marginal_costs"] = ev[key]["speedup_T_hat_over_T_bar_marginal_costs"]
    rep = extra.get("reports", {})
    f16 = rep.get("nested_fp16_cubic16_kahan_levels0to6_2p24")
    if f16:
        out["fp16_cubic16_kahan_levels0to6"] = f16["speedup_T_hat_over_T_bar"]
    pc = rep.get("pconst4096_vs_dyadic_call_levels0to10_2p20")
    if pc:
        out["fp16_cubic16_kahan_levels0to10"] = pc["fp16_cubic16_kahan"]["speedup_T_hat_over_T_bar"]
        out["fp32_pconst4096_levels0to10"] = pc["fp32_pconst"]["speedup_T_hat_over_T_bar"]
        out["fp16_pconst4096_kahan_levels0to10"] = pc["fp16_pconst_kahan"]["speedup_T_hat_over_T_bar"]
    mlp = rep.get("mlp_nested_fp32_levels0to10_2p22")
    if mlp:
        out["fp32_mlp_levels0to10"] = mlp["speedup_T_hat_over_T_bar"]["mlp"]
    return out


def profile_run(what, calibrate_copy):
    """The launches a rocprofv3 summary covers: the dominant kernels exactly as roofline_block
    times them (2 warm-up and 10 timed launches each, nothing else on the device), the
    cooperative kernel of deep single-level calls with few chunks, or the issue-rate probes."""
    import torch

    import paper_2012_09739_amd as M
    torch.cuda.set_device(0)
    M.mlmc_init(0)
    line = {"profile": what}
    if what in ("roofline", "coop"):
        # the timed launches follow about a second of the same kind of load (the binary32
        # level-10 kernel without Kahan updates, a separate entry in a profiler's statistics),
        # as in the full run, where they follow the headline sweep: the shader clock settles first
        call = M.gbm(payoff=M.MLMC_PAYOFF_CALL)
        warm = M.level_args(call, 10, N_PATHS, M.MLMC_FP32, M.MLMC_NESTED_PWL16, 0, SEED)
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < 1.0:
            for _ in range(50):
                M.mlmc_paths(warm)
            torch.cuda.synchronize()
    if what == "roofline":
        for key in ROOFLINE_KERNELS:
            line["roofline" if key == "fp32" else "roofline_" + key] = roofline_block(M, torch, key)
        if calibrate_copy:
            src = torch.empty(256 * 2 ** 20 // 4, dtype=torch.float32, device="cuda").fill_(1.0)
            dst = torch.empty_like(src)
            for _ in range(3):
                dst.copy_(src)
            torch.cuda.synchronize()
            line["copy_calibration_bytes"] = 2 * src.numel() * 4
    elif what == "coop":
        # 256 chunks of 64 paths at level 14 (one per CU): each runs one eight-wave block,
        # seven producer waves ahead of one consumer wave; 2 warm-up and 5 timed calls each
        n, level = 256 * 64, 14
        for tag, prec, mode, kahan in (("nested_fp32_pwl16_kahan", M.MLMC_FP32, M.MLMC_NESTED_PWL16, 1),
                                       ("plain_fp64", M.MLMC_FP64, M.MLMC_EXACT, 0)):
            for _ in range(2):
                M.mlmc_level(call, level, n, prec, mode, kahan, SEED)
            ts = [M.mlmc_level(call, level, n, prec, mode, kahan, SEED)["cost_seconds"] for _ in range(5)]
            line[tag] = {"level": level, "n_paths": n, "call_ms": [t * 1e3 for t in ts],
                         "ns_per_step": statistics.median(ts) * 1e9 / 2 ** level}
    else:
        line["valu_issue_rates"] = valu_rates()
    print(json.dumps(line), flush=True)


def kernel_ms(M, torch, args, reps=10, warm=2):
    """HIP-event times (ms) of the level kernel alone on the current stream: mlmc_paths with no
    per-path outputs launches the level kernel of mlmc_level_ex and nothing else."""
    stream = torch.cuda.current_stream()
    for _ in range(warm):
        M.mlmc_paths(args, stream=stream)
    evs = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        M.mlmc_paths(args, stream=stream)
        e1.record(stream)
        evs.append((e0, e1))
    torch.cuda.synchronize()
    return [e0.elapsed_time(e1) for e0, e1 in evs]


def roofline_block(M, torch, key):
    """Issue roofline of one dominant kernel (alu bound): VALU issue slots per launch over its
    measured duration against the 39.32 T slots/s peak, with the FLOP/s of each precision
    against its vector peak (counts valid for the hashed kernel sources, else null)."""
    k = ROOFLINE_KERNELS[key]
    call = M.gbm(payoff=M.MLMC_PAYOFF_CALL)
    args = M.level_args(call, k["level"], k["n_paths"], getattr(M, k["precision"]), getattr(M, k["mode"]),
                        k["kahan"], SEED)
    times = kernel_ms(M, torch, args)
    ms = sum(times) / len(times)
    steps = k["n_paths"] << k["level"]
    rate = steps / (ms * 1e-3)
    fresh = ISA_SOURCES_SHA256 == sources_sha256(ISA_SOURCES)
    blk = {"bound": "alu", "peak": PEAK_VALU_TOPS, "unit": "T VALU issue slots/s",
           "kernel": k["kernel"], "kernel_ms": ms, "kernel_ms_min": min(times), "launches_timed": len(times),
           "coupled_path_steps_per_s": rate, "traffic": traffic_bytes(key)}
    if fresh:
        achieved = k["slots"] * rate / 1e12
        blk.update(achieved=achieved, frac=achieved / PEAK_VALU_TOPS, slots_per_path_step=k["slots"],
                   valu_instr_per_path_step=k["valu"],
                   flops={p: {"tflops": f * rate / 1e12, "peak_tflops": PEAK_TFLOPS[p],
                              "frac": f * rate / 1e12 / PEAK_TFLOPS[p]} for p, f in k["flops"].items()})
    else:
        blk.update(achieved=None, frac=None, slots_per_path_step=None, valu_instr_per_path_step=None, flops=None)
    return blk


def equal_variance_report(M, E, call):
    """Plain binary64 estimator vs nested binary32 at equal total MLMC variance (Section 3).

    v^_l, c^_l: two-way exact differences in binary64 (the plain estimator's samples);
    v-_l, c-_l: approximate two-way differences in binary32 (independent Philox stream 0);
    V-_l, C-_l: four-way differences (nested samples, stream 1); costs are device times
    per sample from the library's HIP events: of the 2^20-path calls (fixed cost of a call
    included), and marginal (without it, the regime of small tolerances, where the coarse
    levels take many more samples)."""
    rep = {}
    res = {}
    for name, prec, mode, k in (("plain_fp64", M.MLMC_FP64, M.MLMC_EXACT, 0),
                                ("approx_fp32", M.MLMC_FP32, M.MLMC_APPROX_PWL16, 0),
                                ("approx_fp32_kahan", M.MLMC_FP32, M.MLMC_APPROX_PWL16, 1),
                                ("nested_fp32", M.MLMC_FP32, M.MLMC_NESTED_PWL16, 0),
                                ("nested_fp32_kahan", M.MLMC_FP32, M.MLMC_NESTED_PWL16, 1)):
        sde = M.gbm(payoff=M.MLMC_PAYOFF_CALL)
        res[name] = _level_costs(M, sde, LEVELS, N_PATHS, prec, mode, k)
    cost = lambda rows: [r["cost_seconds"] / r["n_paths"] for r in rows]  # noqa: E731
    var = lambda rows, t: [E.level_stats(r["sum"][t], r["sumsq"][t], r["n_paths"])[1] for r in rows]  # noqa: E731
    # per-sample costs without the fixed cost of a call (launch, reduction): what a sample costs
    # when the optimal allocation asks for many more than 2^20 at the coarse levels
    marg = {name: _marginal_costs(M, M.gbm(payoff=M.MLMC_PAYOFF_CALL), LEVELS, prec, mode, k)
            for name, prec, mode, k in (("plain_fp64", M.MLMC_FP64, M.MLMC_EXACT, 0),
                                        ("approx_fp32", M.MLMC_FP32, M.MLMC_APPROX_PWL16, 0),
                                        ("approx_fp32_kahan", M.MLMC_FP32, M.MLMC_APPROX_PWL16, 1),
                                        ("nested_fp32", M.MLMC_FP32, M.MLMC_NESTED_PWL16, 0),
                                        ("nested_fp32_kahan", M.MLMC_FP32, M.MLMC_NESTED_PWL16, 1))}
    v_hat, c_hat = var(res["plain_fp64"], 0), cost(res["plain_fp64"])
    steps = N_PATHS * sum(2 ** l for l in LEVELS)
    rep["fp64_plain_path_steps_per_s"] = steps / sum(r["cost_seconds"] for r in res["plain_fp64"])
    rep["equal_variance"] = {}
    for tag, ap, ne in (("fp32", "approx_fp32", "nested_fp32"), ("fp32_kahan", "approx_fp32_kahan",
                                                                "nested_fp32_kahan")):
        v_bar, c_bar = var(res[ap], 0), cost(res[ap])
        V_bar, C_bar = var(res[ne], 1), cost(res[ne])
        rep["equal_variance"][tag] = {
            "speedup_T_hat_over_T_bar": E.speedup_equal_variance(v_hat, c_hat, v_bar, c_bar, V_bar, C_bar),
            "speedup_T_hat_over_T_bar_marginal_costs": E.speedup_equal_variance(
                v_hat, marg["plain_fp64"], v_bar, marg[ap], V_bar, marg[ne]),
            "marginal_cost_per_sample_s": {"plain_fp64": marg["plain_fp64"], "approx": marg[ap], "nested": marg[ne]},
            "per_level_speedup": [1.0 / f for f in E.per_level_factor(v_hat, c_hat, v_bar, c_bar, V_bar, C_bar)],
            "approx_two_way_path_steps_per_s": steps / sum(r["cost_seconds"] for r in res[ap]),
            "four_way_over_two_way_variance": [V / v for V, v in zip(V_bar, v_hat)],
        }
    return rep


def _marginal_costs(M, sde, levels, prec, mode, kahan, seed=SEED, reps=3):
    """Per-sample device cost without the call's fixed part: (c(4n) - c(n)) / (3n) from the
    library's HIP events (median of `reps` calls each), n = max(2^20, 2^24 / 2^l) so that both
    calls hold several times the resident waves."""
    out = []
    for l in levels:
        n = max(N_PATHS, 2 ** 24 >> l)
        t = []
        for m in (n, 4 * n):
            M.mlmc_level(sde, l, m, prec, mode, kahan, seed)
            c = sorted(M.mlmc_level(sde, l, m, prec, mode, kahan, seed)["cost_seconds"] for _ in range(reps))
            t.append(c[reps // 2])
        out.append((t[1] - t[0]) / (3 * n))
    return out


def _level_costs(M, sde, levels, n, prec, mode, kahan, seed=SEED, reps=3):
    """One level call per level (after a warm one) for the sums, with the median device time of
    `reps` identical calls as its cost (a single small call's time varies by a few us)."""
    rows = []
    for l in levels:
        M.mlmc_level(sde, l, n, prec, mode, kahan, seed)
        calls = [M.mlmc_level(sde, l, n, prec, mode, kahan, seed) for _ in range(reps)]
        r = dict(calls[0])
        r["cost_seconds"] = sorted(c["cost_seconds"] for c in calls)[reps // 2]
        rows.append(r)
    return rows


def reports(M, E, torch, legs=REPORT_LEGS):
    """Report legs of the other workloads (not timed into `value`); `legs` selects them."""
    import numpy as np

    import mlmc_workloads as W
    rep = {}
    var = lambda rows, t: [E.level_stats(r["sum"][t], r["sumsq"][t], r["n_paths"])[1] for r in rows]  # noqa: E731
    mean = lambda rows, t: [E.level_stats(r["sum"][t], r["sumsq"][t], r["n_paths"])[0] for r in rows]  # noqa: E731
    cost = lambda rows: [r["cost_seconds"] / r["n_paths"] for r in rows]  # noqa: E731
    rate = lambda rows: sum(r["path_steps"] for r in rows) / sum(r["cost_seconds"] for r in rows)  # noqa: E731

    from paper_2012_09739_amd import driver as D
    call = M.gbm(payoff=M.MLMC_PAYOFF_CALL)
    adaptive_plain = None
    if "plain" in legs:
        # plain MLMC in binary64, exact inverse CDF: GBM, P = X_T, levels 0..5, 10^4 paths, seed 0
        c1 = W.PLAIN_FP64
        rows = _level_costs(M, M.gbm(), c1["levels"], c1["n_paths"], M.MLMC_FP64, M.MLMC_EXACT, 0)
        rep["plain_fp64_levels0to5_1e4"] = {"mean": mean(rows, 0), "var": var(rows, 0),
                                            "theta_hat": E.plain_estimate([(r["sum"][0], r["n_paths"]) for r in rows]),
                                            "theta_limit_e^mu": math.exp(0.05), "path_steps_per_s": rate(rows)}

    if "fp16" in legs:
        # packed binary16 with Kahan, piecewise cubic, binary64 exact branch: levels 0..6, 2^24 paths
        c3 = W.NESTED_FP16

        def nested_fp16(diag):
            rows = []
            for l in c3["levels"]:
                args = M.level_args(call, l, c3["n_paths"], M.MLMC_FP16, M.MLMC_NESTED_CUBIC16, 1, SEED, diag=diag)
                out = torch.zeros(8, dtype=torch.float64, device="cuda")
                M.mlmc_level_ex(args, out)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                M.mlmc_level_ex(args, out)
                e1.record()
                torch.cuda.synchronize()
                o = out.cpu().numpy()
                rows.append({"sum": list(o[:4]), "sumsq": list(o[4:]), "n_paths": c3["n_paths"],
                             "path_steps": c3["n_paths"] << l, "cost_seconds": e0.elapsed_time(e1) * 1e-3})
            return rows

        # the estimator's samples without the rounding diagnostic (its own binary64 path), and
        # the diagnostic run for the rounding-difference variance
        nested16 = nested_fp16(0)
        diag16 = nested_fp16(1)
        plain = _level_costs(M, call, c3["levels"], c3["n_paths"], M.MLMC_FP64, M.MLMC_EXACT, 0)
        approx16 = _level_costs(M, call, c3["levels"], c3["n_paths"], M.MLMC_FP16, M.MLMC_APPROX_CUBIC16, 1)
        rho = 2.0 ** -11
        bound = [2 ** l * rho ** 2 * (1 + 0.05 * 2.0 ** -l) ** (2 * 2 ** l) * math.exp(0.04) * math.exp(0.14)
                 for l in c3["levels"]]
        rep["nested_fp16_cubic16_kahan_levels0to6_2p24"] = {
            "nested_path_steps_per_s": rate(nested16), "approx_two_way_path_steps_per_s": rate(approx16),
            "plain_fp64_path_steps_per_s": rate(plain),
            "nested_with_rounding_diagnostic_path_steps_per_s": rate(diag16),
            "rounding_variance": var(diag16, 3), "rounding_variance_bound_B_l": bound,
            "four_way_var": var(nested16, 1), "two_way_exact_var": var(nested16, 2),
            "speedup_T_hat_over_T_bar": E.speedup_equal_variance(var(plain, 0), cost(plain), var(approx16, 0),
                                                                 cost(approx16), var(nested16, 1), cost(nested16))}

    if "batch" in legs:
        # batched ragged sweep: 64 GBM parameter sets x levels 0..14, fp16 (l <= 6) / fp32 (l > 6)
        psets = W.batch_parameter_sets(W.BATCH_PSETS, seed=0)
        items = []
        for p, d in enumerate(psets):
            g = M.gbm(mu=d["mu"], sigma=d["sigma"])
            for l in W.BATCH_LEVELS:
                prec = M.MLMC_FP16 if l <= 6 else M.MLMC_FP32
                items.append(M.item(g, l, W.batch_paths(l), prec, 1 if prec == M.MLMC_FP16 else 0, SEED, pset=p))
        out = torch.zeros((len(items), 8), dtype=torch.float64, device="cuda")
        plan = M.mlmc_batch_create(items, M.MLMC_RV_PWL16, out)
        try:
            best = M.mlmc_batch_autotune(plan, 2)
            M.mlmc_batch_run(plan)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(5):
                M.mlmc_batch_run(plan)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / 5
            cfg, n_tasks = M.mlmc_batch_info(plan)
            wave_s = M.mlmc_batch_item_times(plan, len(items))
        finally:
            M.mlmc_batch_destroy(plan)
        steps = sum(it.n_paths << it.level for it in items)
        resident = cfg.waves_per_cu * torch.cuda.get_device_properties(0).multi_processor_count
        # device time attributed to items in proportion to their wavefront time; cost per sample
        share = [w / sum(wave_s) * ms * 1e-3 for w in wave_s]
        per_level = {}
        for it, c in zip(items, share):
            per_level.setdefault(it.level, []).append(c / it.n_paths)
        # the same work as one standalone level call per level (all parameter sets' paths in
        # one launch: the drift and volatility do not change a path's cost), device times
        stand = []
        for l in W.BATCH_LEVELS:
            prec = M.MLMC_FP16 if l <= 6 else M.MLMC_FP32
            r = _level_costs(M, M.gbm(), [l], len(psets) * W.batch_paths(l), prec, M.MLMC_NESTED_PWL16,
                             1 if prec == M.MLMC_FP16 else 0)[0]
            stand.append(r["cost_seconds"] * 1e3)
        rep["batch_64psets_levels0to14"] = {
            "items": len(items), "tasks": n_tasks, "ms_per_sweep": ms, "path_steps": steps,
            "path_steps_per_s": steps / ms * 1e3,
            "standalone_same_work_ms": sum(stand), "standalone_ms_by_level": stand,
            "rate_over_standalone": sum(stand) / ms,
            "autotuned": {"waves_per_cu": best.waves_per_cu, "task_steps": best.task_steps,
                          "priority_level": best.priority_level, "coop_level": best.coop_level,
                          "block_waves": best.block_waves},
            "wave_slot_utilisation": sum(wave_s) / (resident * ms * 1e-3),
            "cost_per_sample_s_by_level": [float(np.mean(per_level[l])) for l in sorted(per_level)]}

    if "mlp" in legs:
        # learned inverse CDF: train on 2^20 pairs, nested four-way levels 0..10 at 2^22 paths vs PWL16
        params = torch.tensor(W.mlp_initial_params(0), dtype=torch.float32, device="cuda")
        t0 = time.perf_counter()
        hist = M.mlmc_mlp_train(M.mlp_cfg(n_pairs=W.MLP_TRAIN_PAIRS), params)
        train_s = time.perf_counter() - t0
        M.mlmc_mlp_load(params)
        words = torch.arange(2 ** 20, dtype=torch.int64, device="cuda").mul(4096).add(2047).to(torch.int32)
        zs = {}
        for rv in (M.MLMC_RV_EXACT, M.MLMC_RV_MLP, M.MLMC_RV_PWL16):
            z = torch.empty(2 ** 20, dtype=torch.float64, device="cuda")
            M.mlmc_icdf(words, 2 ** 20, rv, M.MLMC_FP32, z)
            zs[rv] = z
        torch.cuda.synchronize()
        mlp_rows = _level_costs(M, call, W.MLP_LEVELS, W.MLP_PATHS, M.MLMC_FP32, M.MLMC_NESTED_MLP, 0)
        pwl_rows = _level_costs(M, call, W.MLP_LEVELS, W.MLP_PATHS, M.MLMC_FP32, M.MLMC_NESTED_PWL16, 0)
        mlp_two = _level_costs(M, call, W.MLP_LEVELS, W.MLP_PATHS, M.MLMC_FP32, M.MLMC_APPROX_MLP, 0)
        pwl_two = _level_costs(M, call, W.MLP_LEVELS, W.MLP_PATHS, M.MLMC_FP32, M.MLMC_APPROX_PWL16, 0)
        plain = _level_costs(M, call, W.MLP_LEVELS, W.MLP_PATHS, M.MLMC_FP64, M.MLMC_EXACT, 0)
        # equal-variance time of the nested estimator (Section 3) with each approximate variable
        speed = {tag: E.speedup_equal_variance(var(plain, 0), cost(plain), var(two, 0), cost(two), var(nest, 1),
                                               cost(nest))
                 for tag, two, nest in (("mlp", mlp_two, mlp_rows), ("pwl16", pwl_two, pwl_rows))}
        rep["mlp_nested_fp32_levels0to10_2p22"] = {
            "train_seconds": train_s, "loss_first_epoch": hist[0], "loss_last_epoch": hist[-1],
            "mse_Z_minus_Ztilde": {"mlp": float(((zs[M.MLMC_RV_MLP] - zs[M.MLMC_RV_EXACT]) ** 2).mean()),
                                   "pwl16": float(((zs[M.MLMC_RV_PWL16] - zs[M.MLMC_RV_EXACT]) ** 2).mean())},
            "four_way_var": {"mlp": var(mlp_rows, 1), "pwl16": var(pwl_rows, 1)},
            "nested_path_steps_per_s": {"mlp": rate(mlp_rows), "pwl16": rate(pwl_rows)},
            "nested_rate_mlp_over_pwl16": rate(mlp_rows) / rate(pwl_rows),
            "approx_two_way_path_steps_per_s": {"mlp": rate(mlp_two), "pwl16": rate(pwl_two)},
            "speedup_T_hat_over_T_bar": speed,
            "time_gain_mlp_over_pwl16": speed["mlp"] / speed["pwl16"]}
    if "sweep" in legs:
        # precision-width sweep (Figure 3's question): variance of the rounding difference
        # X-_N - X~_N against the level for bfloat16 (8 bits), binary16 (11) and binary32 (24),
        # without and with Kahan, piecewise cubic, payoff X_T, 2^18 paths per level
        sweep = {}
        gbm_x = M.gbm()
        for name, prec in (("bf16", M.MLMC_BF16), ("fp16", M.MLMC_FP16), ("fp32", M.MLMC_FP32)):
            for k in (0, 1):
                v = []
                for l in range(2, 11):
                    args = M.level_args(gbm_x, l, 2 ** 18, prec, M.MLMC_APPROX_CUBIC16, k, SEED, diag=1)
                    o = torch.zeros(8, dtype=torch.float64, device="cuda")
                    M.mlmc_level_ex(args, o)
                    torch.cuda.synchronize()
                    t = o.cpu().numpy()
                    v.append(E.level_stats(t[3], t[7], 2 ** 18)[1])
                sweep["%s%s" % (name, "_kahan" if k else "")] = v
        rho = {"bf16": 2.0 ** -8, "fp16": 2.0 ** -11, "fp32": 2.0 ** -24}
        sweep["levels"] = list(range(2, 11))
        sweep["bound_B_l"] = {n: [2 ** l * r * r * (1 + 0.05 * 2.0 ** -l) ** (2 * 2 ** l) * math.exp(0.04 + 0.14)
                                  for l in range(2, 11)] for n, r in rho.items()}
        rep["rounding_variance_precision_sweep_cubic_2p18"] = sweep

    if "adaptive" in legs:
        # adaptive MLMC with a per-level precision map from measured costs, against the plain
        # binary64 estimator at the same accuracy (call payoff, eps = 1e-5)
        mixed = D.adaptive_mlmc(call, 1e-5, seed=21)
        adaptive_plain = D.adaptive_mlmc(call, 1e-5, options=(D.PLAIN_FP64,), seed=21)
        with_pc = D.adaptive_mlmc(call, 1e-5, options=D.TABLE_OPTIONS, seed=21)
        rep["adaptive_mlmc_call_eps1e-5_with_pconst"] = {
            "estimate": with_pc["estimate"], "std_error": with_pc["std_error"], "L": with_pc["L"],
            "choice": with_pc["choice"],
            "predicted_speedup_vs_fp64": with_pc["predicted_seconds_single_option"]["fp64"] / with_pc["predicted_seconds"],
            "measured_device_seconds": with_pc["measured_seconds"],
            "measured_device_seconds_one_by_one": with_pc["measured_seconds_one_by_one"]}
        rep["adaptive_mlmc_call_eps1e-5"] = {
            "estimate": mixed["estimate"], "std_error": mixed["std_error"], "L": mixed["L"],
            "choice": mixed["choice"], "predicted_speedup_vs_fp64": mixed["predicted_seconds_single_option"]["fp64"]
            / mixed["predicted_seconds"],
            "measured_device_seconds": mixed["measured_seconds"],
            "plain_fp64_estimate": adaptive_plain["estimate"], "plain_fp64_std_error": adaptive_plain["std_error"],
            "plain_fp64_measured_device_seconds": adaptive_plain["measured_seconds"],
            "measured_speedup_vs_fp64": adaptive_plain["measured_seconds"] / mixed["measured_seconds"],
            "measured_device_seconds_one_by_one": mixed["measured_seconds_one_by_one"],
            "plain_fp64_measured_device_seconds_one_by_one": adaptive_plain["measured_seconds_one_by_one"]}

    if "milstein" in legs:
        # Milstein (Section 4: order-1 strong convergence moves the work to the coarse levels):
        # plain binary64 level variances against Euler-Maruyama's, nested rates, and the adaptive
        # precision map at the same accuracy
        mil = {}
        lv = list(range(0, 11))
        for tag, sch in (("em", M.MLMC_SCHEME_EM), ("milstein", M.MLMC_SCHEME_MILSTEIN)):
            rows = [M.mlmc_level_run(M.level_args(call, l, 2 ** 20, M.MLMC_FP64, M.MLMC_EXACT, 0, SEED, scheme=sch))
                    for l in lv]
            mil["plain_fp64_var_" + tag] = var(rows, 0)
        for tag, prec, mode, k in (("nested_fp32_pwl", M.MLMC_FP32, M.MLMC_NESTED_PWL16, 0),
                                   ("nested_fp16_cubic_kahan", M.MLMC_FP16, M.MLMC_NESTED_CUBIC16, 1),
                                   ("plain_fp64", M.MLMC_FP64, M.MLMC_EXACT, 0)):
            a = M.level_args(call, 10, 2 ** 20, prec, mode, k, SEED, scheme=M.MLMC_SCHEME_MILSTEIN)
            M.mlmc_level_run(a)
            r = M.mlmc_level_run(a)
            mil["level10_path_steps_per_s_" + tag] = r["path_steps"] / r["cost_seconds"]
        mil["levels"] = lv
        m_mixed = D.adaptive_mlmc(call, 1e-5, seed=23, scheme=M.MLMC_SCHEME_MILSTEIN)
        m_plain = D.adaptive_mlmc(call, 1e-5, options=(D.PLAIN_FP64,), seed=23, scheme=M.MLMC_SCHEME_MILSTEIN)
        mil["adaptive_call_eps1e-5"] = {
            "estimate": m_mixed["estimate"], "std_error": m_mixed["std_error"], "L": m_mixed["L"],
            "choice": m_mixed["choice"],
            "predicted_speedup_vs_fp64": m_mixed["predicted_seconds_single_option"]["fp64"]
            / m_mixed["predicted_seconds"],
            "measured_device_seconds": m_mixed["measured_seconds"],
            "plain_fp64_estimate": m_plain["estimate"], "plain_fp64_measured_device_seconds": m_plain["measured_seconds"],
            "measured_speedup_vs_fp64": m_plain["measured_seconds"] / m_mixed["measured_seconds"],
            "measured_device_seconds_one_by_one": m_mixed["measured_seconds_one_by_one"],
            "plain_fp64_measured_device_seconds_one_by_one": m_plain["measured_seconds_one_by_one"],
            "em_plain_fp64_measured_device_seconds": adaptive_plain["measured_seconds"] if adaptive_plain else None}
        rep["milstein_call"] = mil

    if "pconst" in legs:
        # piecewise-constant variable (4096 cells, table lookup) against the piecewise-linear one:
        # four-way variances, rates and the equal-variance speed-up over plain binary64 (call,
        # levels 0..10, 2^20 paths)
        plain_rows = _level_costs(M, call, LEVELS, N_PATHS, M.MLMC_FP64, M.MLMC_EXACT, 0)
        pc = {}
        for tag, prec, approx, nested, k in (
                ("fp32_pconst", M.MLMC_FP32, M.MLMC_APPROX_PCONST4096, M.MLMC_NESTED_PCONST4096, 0),
                ("fp32_pwl16", M.MLMC_FP32, M.MLMC_APPROX_PWL16, M.MLMC_NESTED_PWL16, 0),
                ("fp16_pconst_kahan", M.MLMC_FP16, M.MLMC_APPROX_PCONST4096, M.MLMC_NESTED_PCONST4096, 1),
                ("fp16_cubic16_kahan", M.MLMC_FP16, M.MLMC_APPROX_CUBIC16, M.MLMC_NESTED_CUBIC16, 1)):
            a_rows = _level_costs(M, call, LEVELS, N_PATHS, prec, approx, k)
            n_rows = _level_costs(M, call, LEVELS, N_PATHS, prec, nested, k)
            pc[tag] = {"approx_two_way_path_steps_per_s": rate(a_rows), "nested_path_steps_per_s": rate(n_rows),
                       "four_way_var": var(n_rows, 1),
                       "speedup_T_hat_over_T_bar": E.speedup_equal_variance(
                           var(plain_rows, 0), cost(plain_rows), var(a_rows, 0), cost(a_rows), var(n_rows, 1),
                           cost(n_rows))}
        rep["pconst4096_vs_dyadic_call_levels0to10_2p20"] = pc
    if "marginal" in legs:
        # marginal device cost per coupled path-step of the level kernel alone, (t(4n) - t(n)) /
        # (3 n 2^l), at the coarse levels (where the MLMC allocation puts most samples) and at
        # level 10, from HIP events around mlmc_paths; n = 2^24 / 2^l paths (2^18 at level 10), so
        # that both launches hold several times the resident waves
        marg = {}
        for tag, prec, mode, k in (("nested_fp32_pwl16_kahan", M.MLMC_FP32, M.MLMC_NESTED_PWL16, 1),
                                   ("nested_fp16_cubic16_kahan", M.MLMC_FP16, M.MLMC_NESTED_CUBIC16, 1),
                                   ("plain_fp64", M.MLMC_FP64, M.MLMC_EXACT, 0)):
            row = {}
            for l in (0, 1, 2, 3, 10):
                n = 2 ** 24 >> l if l < 10 else 2 ** 18
                t1 = sum(kernel_ms(M, torch, M.level_args(call, l, n, prec, mode, k, SEED))) / 10
                t4 = sum(kernel_ms(M, torch, M.level_args(call, l, 4 * n, prec, mode, k, SEED))) / 10
                row["level_%d" % l] = {"ms_n": t1, "ms_4n": t4, "n": n,
                                       "ps_per_path_step": (t4 - t1) * 1e9 / (3 * n * 2 ** l)}
            marg[tag] = row
        rep["marginal_cost_per_path_step"] = marg
    if "valu_rates" in legs:
        rep["valu_issue_rates"] = valu_rates()
    np.seterr(all="ignore")
    return rep


def valu_rates(waves=(8, 4), iters=4096):
    """Lane-instructions per CU per ns of single VALU opcodes (libvalurates.so), per resident
    wavefronts per SIMD; divided by the shader clock of the launch (GHz) they are per clock."""
    import ctypes
    path = os.path.join(ROOT, "paper_2012_09739_amd", "libvalurates.so")
    if not os.path.exists(path):
        raise RuntimeError("libvalurates.so is not built: run python -m paper_2012_09739_amd.build")
    lib = ctypes.CDLL(path)
    lib.valu_rate.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint32, ctypes.POINTER(ctypes.c_double),
                              ctypes.POINTER(ctypes.c_double)]
    out = {}
    for w in waves:
        row = {}
        for op, name in enumerate(VALU_OPS):
            r, ms = ctypes.c_double(), ctypes.c_double()
            rc = lib.valu_rate(op, w, iters, ctypes.byref(r), ctypes.byref(ms))
            if rc != 0:
                raise RuntimeError("valu_rate(%s) failed: %d" % (name, rc))
            row[name] = {"lane_instr_per_cu_per_ns": r.value, "kernel_ms": ms.value}
        out["waves_per_simd_%d" % w] = row
    return out


CPU_SINGLE_PATHS = 2 ** 15     # paths per level, one process
CPU_POOL_PATHS = 2 ** 19       # paths per level over the worker pool
CPU_TASK_PATHS = 2 ** 15       # paths per worker task
CPU_MAX_WORKERS = 16           # the host share of one GPU


def _oracle_task(task):
    """One bounded piece of the CPU baseline: oracle level sums over a path range."""
    import mlmc_workloads as W
    from oracle import fp, mlmc
    level, offset, n = task
    mlmc.level_sums(level, n, W.GBM_CALL, path_offset=offset, rv_mode=mlmc.RV_PWL, precision=fp.FP32,
                    nested=True, kahan=True, seed=SEED, stream=1)
    return n * 2 ** level


def cpu_baseline():
    """The CPU oracle (float64 NumPy with binary32 emulation) on bounded samples of the
    same workload (nested binary32 PWL16 with Kahan, levels 0..10): one process on
    CPU_SINGLE_PATHS paths per level, then a pool of worker processes (at most the 16
    cores of one GPU's host share) on CPU_POOL_PATHS paths per level."""
    import multiprocessing as mp

    t0 = time.perf_counter()
    steps1 = sum(_oracle_task((l, 0, CPU_SINGLE_PATHS)) for l in LEVELS)
    dt1 = time.perf_counter() - t0

    workers = max(1, min(CPU_MAX_WORKERS, os.cpu_count() or 1))
    tasks = [(l, off, CPU_TASK_PATHS) for l in reversed(LEVELS) for off in range(0, CPU_POOL_PATHS, CPU_TASK_PATHS)]
    with mp.get_context("spawn").Pool(workers) as pool:
        pool.map(_oracle_task, [(0, 0, 64)] * workers, chunksize=1)  # start-up and imports, untimed
        t0 = time.perf_counter()
        steps = sum(pool.imap_unordered(_oracle_task, tasks, chunksize=1))
        dt = time.perf_counter() - t0
    return {"value": steps / dt, "unit": "coupled path-steps/s", "cores": workers, "kind": "oracle",
            "sample": "nested fp32 PWL16 Kahan, levels 0..10, 2^%d paths/level" % (CPU_POOL_PATHS.bit_length() - 1),
            "sample_path_steps": steps, "sample_seconds": dt,
            "single_core_value": steps1 / dt1, "single_core_sample_paths_per_level": CPU_SINGLE_PATHS,
            "single_core_seconds": dt1, "host_cpu_count": os.cpu_count(), "host_cpu_model": _cpu_model(),
            "worker_cap": CPU_MAX_WORKERS}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


if __name__ == "__main__":
    main()
