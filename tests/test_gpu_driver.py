"""GPU test of the adaptive MLMC driver: with X_T as the payoff the level-L Euler scheme
with exact variables has E[X_N] = X0 (1 + mu 2^-L)^(2^L) exactly (binary64 rounding aside),
and every per-level option (plain binary64, or nested binary32 / binary16 with the four-way
correction) has the same expectation, so the mixed estimator must land within a few
standard errors of that value.  The Milstein factor 1 + mu delta + sigma dW +
sigma^2 (dW^2 - delta) / 2 has the same expectation 1 + mu delta, so the same value holds for
the Milstein levels."""

import math

import pytest

import paper_2012_09739_amd as M
from paper_2012_09739_amd import driver as D

pytestmark = pytest.mark.gpu


def test_adaptive_mixture_is_unbiased_and_meets_the_target():
    eps = 1e-4
    out = D.adaptive_mlmc(M.gbm(), eps, n_pilot=1 << 16, seed=11)
    L = out["L"]
    assert 3 <= L <= 8, L
    exact = (1.0 + 0.05 * 2.0 ** -L) ** (2 ** L)
    assert abs(out["estimate"] - exact) <= 4.0 * out["std_error"], (out["estimate"], exact, out["std_error"])
    assert out["std_error"] <= eps / math.sqrt(2) * 1.25
    assert len(out["choice"]) == L + 1
    assert out["predicted_seconds"] <= min(out["predicted_seconds_single_option"].values()) * (1 + 1e-12)
    assert out["measured_seconds"] > 0


def test_plain_only_driver_matches_the_same_value():
    eps = 2e-4
    out = D.adaptive_mlmc(M.gbm(), eps, options=(D.PLAIN_FP64,), n_pilot=1 << 16, seed=12)
    L = out["L"]
    exact = (1.0 + 0.05 * 2.0 ** -L) ** (2 ** L)
    assert set(out["choice"]) == {"fp64"}
    assert abs(out["estimate"] - exact) <= 4.0 * out["std_error"]


def test_milstein_adaptive_mixture_is_unbiased():
    eps = 1e-4
    out = D.adaptive_mlmc(M.gbm(), eps, n_pilot=1 << 16, seed=13, scheme=M.MLMC_SCHEME_MILSTEIN)
    L = out["L"]
    exact = (1.0 + 0.05 * 2.0 ** -L) ** (2 ** L)
    assert abs(out["estimate"] - exact) <= 4.0 * out["std_error"], (out["estimate"], exact, out["std_error"])
    assert out["std_error"] <= eps / math.sqrt(2) * 1.25
    assert out["predicted_seconds"] <= min(out["predicted_seconds_single_option"].values()) * (1 + 1e-12)


def test_mixture_with_table_lookup_options_is_unbiased():
    eps = 1e-4
    out = D.adaptive_mlmc(M.gbm(), eps, options=D.TABLE_OPTIONS, n_pilot=1 << 16, seed=17)
    L = out["L"]
    exact = (1.0 + 0.05 * 2.0 ** -L) ** (2 ** L)
    assert abs(out["estimate"] - exact) <= 4.0 * out["std_error"], (out["estimate"], exact, out["std_error"])
    assert out["std_error"] <= eps / math.sqrt(2) * 1.25
    assert set(out["predicted_seconds_single_option"]) == {o.name for o in D.TABLE_OPTIONS}
