"""Seeded synthetic workloads shared by the tests, bench.py and smoke().

Holds none of the method's arithmetic: only the problem sizes of the five workload
configurations and the seeded draws of inputs (GBM parameter sets, MLP initial weights),
which both the GPU library and the CPU oracle receive as plain inputs.

The paper's experiments use geometric Brownian motion with mu = 0.05, sigma = 0.2,
X_0 = 1 (Section 2.2), T = 1, and P(X) = X (Section 3); there is no dataset.
"""

import numpy as np

GBM = dict(mu=0.05, sigma=0.2, x0=1.0, T=1.0, payoff=0, strike=1.0)
GBM_CALL = dict(GBM, payoff=1)

# plain MLMC, binary64, exact inverse CDF: levels 0..5, 10^4 paths per level, seed 0
PLAIN_FP64 = dict(name="plain-fp64-exact-gbm", levels=list(range(6)), n_paths=10 ** 4, seed=0, sde=GBM)
# nested four-way, binary32, piecewise linear on 16 dyadic intervals, call payoff, with and
# without Kahan: levels 0..10, 2^20 paths per level
NESTED_FP32 = dict(name="nested-fp32-pwl16-call", levels=list(range(11)), n_paths=2 ** 20, seed=0,
                   sde=GBM_CALL, kahan=(0, 1))
# packed half2 path arithmetic with Kahan, piecewise cubic, binary64 exact branch:
# levels 0..6, 2^24 paths per level, rounding-error diagnostic
NESTED_FP16 = dict(name="nested-fp16-cubic16-kahan", levels=list(range(7)), n_paths=2 ** 24, seed=0,
                   sde=GBM_CALL, kahan=(1,))
# batched ragged sweep: 64 GBM parameter sets, levels 0..14, N_l = max(256, round(2^(22-1.5 l)))
BATCH_LEVELS = list(range(15))
BATCH_PSETS = 64
# learned inverse CDF: 2^20 training pairs; nested four-way on levels 0..10 at 2^22 paths
MLP_TRAIN_PAIRS = 2 ** 20
MLP_LEVELS = list(range(11))
MLP_PATHS = 2 ** 22


def batch_paths(level):
    return max(256, int(round(2.0 ** (22 - 1.5 * level))))


def batch_parameter_sets(n=BATCH_PSETS, seed=0):
    """n GBM parameter sets: mu ~ U[0, 0.1], sigma ~ U[0.1, 0.5], X0 = 1, T = 1."""
    rng = np.random.default_rng(seed)
    mu = rng.uniform(0.0, 0.1, n)
    sigma = rng.uniform(0.1, 0.5, n)
    return [dict(mu=float(m), sigma=float(s), x0=1.0, T=1.0, payoff=0, strike=1.0) for m, s in zip(mu, sigma)]


def mlp_initial_params(seed=0):
    """Initial weights of the 1-16-16-1 hard-tanh network: first-layer slopes |W1| ~ U[2, 6]
    with random signs and biases b1 ~ U(-1, 1) |W1|, so that every unit's two kinks
    (W1 x + b1 = +-1) fall near the input range [-1, 1]; W2 ~ U(-1, 1); output weights at
    the Glorot-uniform scale; zero b2, b3."""
    rng = np.random.default_rng(seed)
    w1 = rng.uniform(2.0, 6.0, 16) * rng.choice([-1.0, 1.0], 16)
    b1 = rng.uniform(-1.0, 1.0, 16) * np.abs(w1)
    w2 = rng.uniform(-1.0, 1.0, 256)
    w3 = rng.uniform(-1, 1, 16) * np.sqrt(6 / 17)
    return np.concatenate([w1, b1, w2, np.zeros(16), w3, [0.0]]).astype(np.float64)


def sampled_paths(n_paths, k=64, seed=1):
    """k path indices spread over [0, n_paths), always including the first and last."""
    rng = np.random.default_rng(seed)
    idx = set(rng.integers(0, n_paths, max(k - 2, 0)).tolist()) | {0, n_paths - 1}
    return np.array(sorted(idx), dtype=np.int64)
