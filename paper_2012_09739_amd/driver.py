"""Adaptive MLMC with a per-level precision map chosen from measured device costs.

Section 3 writes each level correction of the nested estimator as an approximate two-way
difference plus a four-way correction; a level may instead use the plain exact two-way
difference.  Every option has the same expectation E[P^_l - P^_{l-1}] (the four-way term
removes the approximation's bias exactly), so any per-level mixture of options is an
unbiased estimator of E[P^_L].  With optimal sample counts the cost of reaching mean
squared error eps^2 (variance eps^2 / 2, bias at most eps / sqrt 2) is

    T = 2 eps^-2 (sum_l a_l)^2,   a_l = sqrt(v^_l c^_l)                      (plain)
                                  a_l = sqrt(v-_l c-_l) + sqrt(V-_l C-_l)      (nested)

(Section 3's T^ and T-), so with costs proportional to the sample counts the cheapest mixture
takes at every level the option with the smallest a_l.  The number of samples of each term j
is m_j = 2 eps^-2 sqrt(v_j / c_j) sum_k sqrt(v_k c_k) over all terms of all levels.  A level
call also has a fixed device cost f (launch, table staging, reduction) that the per-sample
model leaves out; a nested option pays it twice per level (its two terms are two calls), which
at large tolerances, where the calls are small, can outweigh what its cheaper samples save.
The choice therefore minimises T + sum of the chosen calls' f: it starts from the per-level
minimisers of a_l (and from every single option used at all levels) and changes one level at
a time while the total falls.

Levels are added until Giles' weak-error test holds: with alpha = 1 (the weak order of
both Euler-Maruyama and Milstein), max(|E d_L|, |E d_{L-1}| / 2) / (2^alpha - 1) <= eps / sqrt 2,
d_l the exact two-way difference.  Every level of one run uses the same scheme; with
Milstein (order-1 strong convergence) the level variances fall as 4^-l instead of 2^-l and
the work moves to the coarse levels, where the low-precision options are cheapest
(Section 4).  Every sample comes from the level calls of the C-ABI; the arithmetic here
is on a few numbers per level.  Pilot and final samples use different Philox keys.
"""

import math
from dataclasses import dataclass, field

from . import mlmc as M
from .estimators import level_stats

ALPHA = 1.0  # weak order of Euler-Maruyama


@dataclass(frozen=True)
class Option:
    """One way of sampling a level correction."""
    name: str
    precision: int          # MLMC_FP64 (plain, exact variables) or the approximate pair's
    rv: int = M.MLMC_RV_EXACT
    kahan: int = 0

    @property
    def nested(self):
        return self.rv != M.MLMC_RV_EXACT


PLAIN_FP64 = Option("fp64", M.MLMC_FP64)
NESTED_FP32 = Option("fp32-pwl", M.MLMC_FP32, M.MLMC_RV_PWL16, 0)
NESTED_FP32_KAHAN = Option("fp32-pwl-kahan", M.MLMC_FP32, M.MLMC_RV_PWL16, 1)
NESTED_FP16_KAHAN = Option("fp16-cubic-kahan", M.MLMC_FP16, M.MLMC_RV_CUBIC16, 1)
NESTED_FP32_PCONST = Option("fp32-pconst", M.MLMC_FP32, M.MLMC_RV_PCONST4096, 0)
NESTED_FP16_PCONST_KAHAN = Option("fp16-pconst-kahan", M.MLMC_FP16, M.MLMC_RV_PCONST4096, 1)
DEFAULT_OPTIONS = (PLAIN_FP64, NESTED_FP32, NESTED_FP32_KAHAN, NESTED_FP16_KAHAN)
TABLE_OPTIONS = DEFAULT_OPTIONS + (NESTED_FP32_PCONST, NESTED_FP16_PCONST_KAHAN)


@dataclass
class LevelPilot:
    """Pilot statistics of one level: per option the variances and costs per sample of its
    terms (plain: [(v^, c^)]; nested: [(v-, c-), (V-, C-)]) and the exact two-way mean."""
    level: int
    terms: dict = field(default_factory=dict)
    fixed: dict = field(default_factory=dict)  # per option: the fixed device cost of each term's call
    mean_exact: float = 0.0


# ---- pure arithmetic (CPU-testable) ---------------------------------------------------------

def cost_weight(terms):
    """a_l of an option: sum over its terms of sqrt(v c)."""
    return math.fsum(math.sqrt(v * c) for v, c in terms)


def choose(pilot):
    """Name of the option with the smallest a_l at this level."""
    return min(pilot.terms, key=lambda k: cost_weight(pilot.terms[k]))


def total_time(pilots, choice, eps):
    """Predicted device time of a per-level choice: the per-sample model T plus the fixed cost
    of every call it makes (one per term of each level's option)."""
    flat = [vc for p, name in zip(pilots, choice) for vc in p.terms[name]]
    fixed = math.fsum(f for p, name in zip(pilots, choice) for f in p.fixed.get(name, ()))
    return predicted_time(flat, eps) + fixed


def choose_levels(pilots, eps):
    """Per-level option names minimising total_time: the best of the per-level a_l minimisers
    and of every single option, then single-level changes while the total falls."""
    names = list(pilots[0].terms)
    starts = [[choose(p) for p in pilots]] + [[n] * len(pilots) for n in names]
    best = list(min(starts, key=lambda ch: total_time(pilots, ch, eps)))
    cur = total_time(pilots, best, eps)
    improved = True
    while improved:
        improved = False
        for l in range(len(pilots)):
            for name in names:
                if name == best[l]:
                    continue
                trial = best[:l] + [name] + best[l + 1:]
                t = total_time(pilots, trial, eps)
                if t < cur * (1.0 - 1e-12):
                    best, cur, improved = trial, t, True
    return best


def allocate(terms, eps):
    """Optimal sample counts for a flat list of (v, c) terms at mean squared error eps^2."""
    total = math.fsum(math.sqrt(v * c) for v, c in terms)
    return [max(2, math.ceil(2.0 / eps ** 2 * math.sqrt(v / c) * total)) for v, c in terms]


def predicted_time(terms, eps):
    """T = 2 eps^-2 (sum sqrt(v c))^2 for a flat list of (v, c) terms."""
    return 2.0 / eps ** 2 * math.fsum(math.sqrt(v * c) for v, c in terms) ** 2


def weak_converged(means, eps, alpha=ALPHA):
    """Giles' test on the exact two-way means of levels 0..L (needs L >= 2)."""
    if len(means) < 3:
        return False
    rem = max(abs(means[-1]), abs(means[-2]) / 2.0 ** alpha) / (2.0 ** alpha - 1.0)
    return rem <= eps / math.sqrt(2.0)


# ---- sampling through the C-ABI ------------------------------------------------------------

def _stats(r, term):
    mean, var = level_stats(r["sum"][term], r["sumsq"][term], r["n_paths"])
    return mean, var


def _marginal(call, n):
    """Run n and then 2n samples; returns the 2n-sample result, the device time per extra
    sample c = (t(2n) - t(n)) / n, which leaves out the fixed cost of a call (launch,
    reduction), and that fixed cost t(n) - n c (at least 0)."""
    r1 = call(n)
    r2 = call(2 * n)
    extra = r2["cost_seconds"] - r1["cost_seconds"]
    c = max(extra, 0.05 * r2["cost_seconds"]) / n
    return r2, c, max(0.0, r1["cost_seconds"] - c * n)


def _level(sde, level, n, precision, rv_mode, kahan, seed, scheme):
    """One synchronous level call (Philox stream 1 for nested modes, 0 otherwise)."""
    return M.mlmc_level_run(M.level_args(sde, level, n, precision, rv_mode, kahan, seed, scheme=scheme))


def pilot_level(sde, level, options, n, seed, scheme=M.MLMC_SCHEME_EM):
    """Pilot runs of every option at one level: variances from 2n samples, device costs per
    sample as marginal costs (after a warm call, so that no first-launch cost enters)."""
    p = LevelPilot(level)
    for opt in options:
        if not opt.nested:
            _level(sde, level, 1024, opt.precision, M.MLMC_EXACT, 0, seed, scheme)
            r, c, f = _marginal(lambda k: _level(sde, level, k, opt.precision, M.MLMC_EXACT, 0, seed, scheme), n)
            m, v = _stats(r, 0)
            p.terms[opt.name] = [(v, c)]
            p.fixed[opt.name] = [f]
            p.mean_exact = m
        else:
            approx, nested = opt.rv, opt.rv + 4
            _level(sde, level, 1024, opt.precision, approx, opt.kahan, seed, scheme)
            _level(sde, level, 1024, opt.precision, nested, opt.kahan, seed, scheme)
            r, c, f = _marginal(lambda k: _level(sde, level, k, opt.precision, approx, opt.kahan, seed, scheme), n)
            _, v = _stats(r, 0)
            r, C, F = _marginal(lambda k: _level(sde, level, k, opt.precision, nested, opt.kahan, seed, scheme), n)
            _, V = _stats(r, 1)
            p.terms[opt.name] = [(v, c), (V, C)]
            p.fixed[opt.name] = [f, F]
            if not any(not o.nested for o in options):
                p.mean_exact = _stats(r, 2)[0]
    return p


def _term_call(sde, level, opt, term_index, n, seed, scheme=M.MLMC_SCHEME_EM):
    """Arguments of the level call that draws n samples of one term of one option, and the
    index of that term in the call's result."""
    if not opt.nested:
        mode, kahan, t = M.MLMC_EXACT, 0, 0
    elif term_index == 0:
        mode, kahan, t = opt.rv, opt.kahan, 0
    else:
        mode, kahan, t = opt.rv + 4, opt.kahan, 1
    return M.level_args(sde, level, n, opt.precision, mode, kahan, seed, scheme=scheme), t


def _run_term(sde, level, opt, term_index, n, seed, scheme=M.MLMC_SCHEME_EM):
    """n samples of one term of one option; returns (sum, sum of squares, n, device seconds)."""
    args, t = _term_call(sde, level, opt, term_index, n, seed, scheme)
    r = M.mlmc_level_run(args)
    return r["sum"][t], r["sumsq"][t], n, r["cost_seconds"]


def adaptive_mlmc(sde, eps, options=DEFAULT_OPTIONS, *, l_min=2, l_max=14, n_pilot=2 ** 19, seed=0,
                  max_samples=2 ** 32, scheme=M.MLMC_SCHEME_EM, concurrent=True):
    """Adaptive MLMC to root-mean-square error eps with a per-level choice among options.

    Returns a dict: estimate, its standard error, L, per-level choice, samples per term,
    the predicted device time (per-sample model plus the calls' fixed costs) of the chosen
    mixture and of each single option used at every level (the plain binary64 estimator among
    them), and the measured device time of the final sampling (pilot runs excluded).  concurrent: the final sampling is one level set
    (mlmc_level_set_run: every term's call issued together, deep levels first, over several
    streams) and the measured time is its span; otherwise the calls run one after another
    and the measured time is the sum of their device times, each with its fixed launch and
    reduction cost.  The samples, and so
    the estimate, are the same either way."""
    by_name = {o.name: o for o in options}
    pilots = []
    level = 0
    while True:
        pilots.append(pilot_level(sde, level, options, n_pilot, seed, scheme))
        if level >= l_min and weak_converged([p.mean_exact for p in pilots], eps):
            break
        if level == l_max:
            break
        level += 1
    L = level
    choice = choose_levels(pilots, eps)
    flat, where = [], []
    for l, (p, name) in enumerate(zip(pilots, choice)):
        for j, vc in enumerate(p.terms[name]):
            flat.append(vc)
            where.append((l, name, j))
    counts = allocate(flat, eps)
    if max(counts) > max_samples:
        raise ValueError("eps too small for max_samples")
    final_seed = seed + 1
    sums = {}
    device_s = 0.0
    one_by_one = None
    if concurrent:
        calls = [_term_call(sde, l, by_name[name], j, n, final_seed, scheme) for (l, name, j), n in zip(where, counts)]
        results, device_s = M.mlmc_level_set_run([a for a, _ in calls])
        for (l, _, j), n, (_, t), r in zip(where, counts, calls, results):
            sums[(l, j)] = (r["sum"][t], r["sumsq"][t], n)
        # the same calls once more, one after another, for the device time without overlap
        one_by_one = math.fsum(M.mlmc_level_run(a)["cost_seconds"] for a, _ in calls)
    else:
        for (l, name, j), n in zip(where, counts):
            s, q, m, t = _run_term(sde, l, by_name[name], j, n, final_seed, scheme)
            sums[(l, j)] = (s, q, m)
            device_s += t
    estimate, var = 0.0, 0.0
    parts = []
    for (l, j), (s, q, m) in sorted(sums.items()):
        mean, v = level_stats(s, q, m)
        parts.append(mean)
        var += v / m
    estimate = math.fsum(parts)
    single = {o.name: total_time(pilots, [o.name] * len(pilots), eps) for o in options}
    return {"estimate": estimate, "std_error": math.sqrt(var), "L": L, "choice": choice,
            "samples": {"%d/%s/%d" % w: n for w, n in zip(where, counts)},
            "predicted_seconds": total_time(pilots, choice, eps), "predicted_seconds_single_option": single,
            "predicted_seconds_per_sample_model": predicted_time(flat, eps),
            "per_level_fixed_seconds": [dict(p.fixed) for p in pilots],
            "measured_seconds": device_s, "measured_seconds_one_by_one": one_by_one,
            "per_level_a": [{k: cost_weight(v) for k, v in p.terms.items()} for p in pilots]}
