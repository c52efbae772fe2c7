"""Host logic of the adaptive MLMC driver (per-level option choice, optimal allocation,
weak-error test), with a synthetic sampler standing in for the level calls: its sums are
exact functions of prescribed means, variances and costs, so the driver's arithmetic can be
checked against closed forms without a GPU."""

import math

import pytest

import paper_2012_09739_amd as M
from paper_2012_09739_amd import driver as D


def test_allocate_meets_the_variance_target_at_the_predicted_cost():
    terms = [(0.04, 1e-9), (4e-4, 2e-9), (2e-4, 4e-9), (1e-5, 3e-9), (1e-7, 8e-9)]
    eps = 1e-3
    m = D.allocate(terms, eps)
    var = math.fsum(v / n for (v, _), n in zip(terms, m))
    cost = math.fsum(c * n for (_, c), n in zip(terms, m))
    assert var <= eps ** 2 / 2 * (1 + 1e-12)
    assert var >= eps ** 2 / 2 * 0.999          # ceil only rounds counts up slightly
    assert cost == pytest.approx(D.predicted_time(terms, eps), rel=1e-3)
    # Lagrange: m_j = ceil(K s_j) with s_j = sqrt(v_j / c_j) and one K for all terms
    s_j = [math.sqrt(v / c) for v, c in terms]
    K = 2.0 / eps ** 2 * math.fsum(math.sqrt(v * c) for v, c in terms)
    assert all(K * sj <= n < K * sj + 1 for sj, n in zip(s_j, m))


def test_choice_takes_the_smallest_cost_weight():
    p = D.LevelPilot(3, terms={"a": [(1e-4, 4e-9)], "b": [(1e-4, 1e-9), (1e-8, 4e-9)], "c": [(1e-3, 1e-9)]})
    assert D.cost_weight(p.terms["b"]) == pytest.approx(math.sqrt(1e-13) + math.sqrt(4e-17))
    assert D.choose(p) == "b"


@pytest.mark.parametrize("K,eps,L_expected", [(1e-2, 1e-3, 4), (1e-2, 1e-4, 8)])
def test_weak_error_test(K, eps, L_expected):
    # means d_l = K 2^-l: converged at the first L >= 2 with K 2^-L <= eps / sqrt 2
    L = next(L for L in range(2, 40) if D.weak_converged([K * 2.0 ** -l for l in range(L + 1)], eps))
    assert L == L_expected
    assert K * 2.0 ** -L <= eps / math.sqrt(2) < K * 2.0 ** -(L - 1)


class FakeLevels:
    """Stands in for mlmc_level_run: sums of n samples equal n * mean and the sums of squares
    n * (var + mean^2), so level_stats returns the prescribed mean and (n/(n-1)) var."""

    def __init__(self, mu=0.05, fixed=0.0):
        self.calls = []
        self.schemes = set()
        self.mu = mu
        self.fixed = fixed  # device seconds every call costs besides its samples

    def moments(self, level, precision, mode):
        d = 1e-2 * 2.0 ** -level
        v_exact = 0.04 if level == 0 else 1e-3 * 2.0 ** -level
        base = {M.MLMC_FP64: 8e-9, M.MLMC_FP32: 2e-9, M.MLMC_FP16: 1e-9}[precision] * 2 ** level
        if mode == M.MLMC_EXACT:
            return [(d, v_exact)], base
        approx = mode in (M.MLMC_RV_PWL16, M.MLMC_RV_CUBIC16)
        if approx:
            return [(d * 0.99, v_exact)], base
        return [(d * 0.99, v_exact), (d * 0.01, 1e-8 * 2.0 ** -level), (d, v_exact)], base + 8e-9 * 2 ** level

    def __call__(self, args):
        level, n, precision, mode = args.level, args.n_paths, args.precision, args.rv_mode
        kahan, seed = args.kahan, args.seed
        self.schemes.add(args.scheme)
        self.calls.append((level, n, precision, mode, kahan, seed))
        terms, c = self.moments(level, precision, mode)
        s, q = [math.nan] * 4, [math.nan] * 4
        for k, (mean, var) in enumerate(terms):
            s[k] = n * mean
            q[k] = n * (var + mean * mean)
        return {"sum": s, "sumsq": q, "n_paths": n, "path_steps": n << level, "cost_seconds": self.fixed + c * n}

    def set_run(self, args_list):
        """Stands in for mlmc_level_set_run: the calls as if run side by side."""
        res = [self(a) for a in args_list]
        return res, max(r["cost_seconds"] for r in res)


def patch(monkeypatch, fake):
    monkeypatch.setattr(D.M, "mlmc_level_run", fake)
    monkeypatch.setattr(D.M, "mlmc_level_set_run", fake.set_run)


def test_driver_orchestration_with_synthetic_levels(monkeypatch):
    fake = FakeLevels()
    patch(monkeypatch, fake)
    eps = 1e-3
    out = D.adaptive_mlmc(M.gbm(), eps, n_pilot=1 << 16)
    L = out["L"]
    assert L == 4                                     # 1e-2 2^-L <= eps / sqrt 2
    # the estimate is the sum of the prescribed level means whatever the choice per level
    assert out["estimate"] == pytest.approx(math.fsum(1e-2 * 2.0 ** -l for l in range(L + 1)), rel=1e-12)
    # every level's choice minimises a_l, and the mixture is never predicted slower than a
    # single option used at every level
    for l, name in enumerate(out["choice"]):
        a = out["per_level_a"][l]
        assert a[name] == min(a.values())
    assert out["predicted_seconds"] <= min(out["predicted_seconds_single_option"].values()) * (1 + 1e-12)
    # with these costs the nested binary16 option wins at every level and the plain one loses
    assert set(out["choice"]) == {"fp16-cubic-kahan"}
    # pilot and final samples use different Philox keys
    assert {c[-1] for c in fake.calls} == {0, 1}
    assert out["std_error"] <= eps / math.sqrt(2) * 1.01
    assert fake.schemes == {M.MLMC_SCHEME_EM}


def test_total_time_adds_the_fixed_cost_of_every_call():
    p0 = D.LevelPilot(0, terms={"plain": [(1e-2, 8e-9)], "nested": [(1e-2, 2e-9), (1e-6, 1e-8)]},
                      fixed={"plain": [2e-5], "nested": [2e-5, 3e-5]})
    p1 = D.LevelPilot(1, terms={"plain": [(1e-3, 1.6e-8)], "nested": [(1e-3, 4e-9), (1e-7, 2e-8)]},
                      fixed={"plain": [2e-5], "nested": [2e-5, 3e-5]})
    eps = 1e-3
    for choice, fixed in ((["plain", "plain"], 4e-5), (["nested", "plain"], 7e-5), (["nested", "nested"], 1e-4)):
        flat = [vc for p, n in zip((p0, p1), choice) for vc in p.terms[n]]
        assert D.total_time([p0, p1], choice, eps) == pytest.approx(D.predicted_time(flat, eps) + fixed, rel=1e-14)


@pytest.mark.parametrize("eps,expect_plain", [(3e-2, True), (1e-4, False)])
def test_choice_weighs_the_fixed_cost_of_a_call(monkeypatch, eps, expect_plain):
    # nested options make two calls per level: at a large tolerance (few samples) the calls'
    # fixed cost decides and the plain estimator wins everywhere; at a small one the per-sample
    # costs decide and the cheapest nested option does
    fake = FakeLevels(fixed=2e-5)
    patch(monkeypatch, fake)
    out = D.adaptive_mlmc(M.gbm(), eps, n_pilot=1 << 12)
    if expect_plain:
        assert set(out["choice"]) == {"fp64"}
    else:
        assert set(out["choice"]) == {"fp16-cubic-kahan"}
    assert out["predicted_seconds"] <= min(out["predicted_seconds_single_option"].values()) * (1 + 1e-12)
    for l, f in enumerate(out["per_level_fixed_seconds"]):
        assert f["fp64"] == [pytest.approx(2e-5, rel=1e-9)]
        assert f["fp16-cubic-kahan"] == [pytest.approx(2e-5, rel=1e-9)] * 2


def test_driver_passes_the_scheme_to_every_call(monkeypatch):
    fake = FakeLevels()
    patch(monkeypatch, fake)
    D.adaptive_mlmc(M.gbm(), 1e-3, n_pilot=1 << 10, scheme=M.MLMC_SCHEME_MILSTEIN)
    assert fake.schemes == {M.MLMC_SCHEME_MILSTEIN}


def test_concurrent_final_sampling_draws_the_same_samples(monkeypatch):
    fake = FakeLevels()
    patch(monkeypatch, fake)
    a = D.adaptive_mlmc(M.gbm(), 1e-3, n_pilot=1 << 12, concurrent=True)
    final_a = [c for c in fake.calls if c[-1] == 1]
    fake.calls.clear()
    b = D.adaptive_mlmc(M.gbm(), 1e-3, n_pilot=1 << 12, concurrent=False)
    final_b = [c for c in fake.calls if c[-1] == 1]
    assert sorted(final_a) == sorted(final_b * 2)    # the set, then the same calls timed one by one
    assert a["estimate"] == b["estimate"] and a["std_error"] == b["std_error"]
    # one set: the span is the longest call; one after another: the sum of the calls
    costs = [fake(D._term_call(M.gbm(), l, D.NESTED_FP16_KAHAN, j, n, 1)[0])["cost_seconds"]
             for (l, j), n in ((tuple(int(x) for x in k.split("/")[::2]), n) for k, n in b["samples"].items())]
    assert a["measured_seconds"] == pytest.approx(max(costs))
    assert b["measured_seconds"] == pytest.approx(sum(costs))
    assert a["measured_seconds_one_by_one"] == pytest.approx(sum(costs))
