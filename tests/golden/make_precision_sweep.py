"""Writes tests/golden/precision_sweep_oracle.json from the CPU oracle alone: the variance of
the rounding difference X-_N - X~_N (Lemma 2.6's quantity; term 3 of a level call) for
7-, 10-, 16- and 23-bit mantissas (bfloat16, binary16, the 17-significant-bit emulation and
binary32), without and with Kahan compensation, piecewise cubic variables, P = X_T, GBM
mu = 0.05, sigma = 0.2, levels 2..8, 4096 paths per level, seed 2 -- the precision-width
experiments around Figure 3, including the width no GPU format provides.

Run from the repository root:  python tests/golden/make_precision_sweep.py
"""

import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import fp, mlmc  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
GBM = dict(mu=0.05, sigma=0.2, x0=1.0, T=1.0, payoff=mlmc.PAYOFF_X, strike=1.0)
LEVELS = list(range(2, 9))
PATHS = 4096


def main():
    out = {"citation": "Section 2.2, Lemma 2.6 and the precision experiments around Figure 3: "
                       "variance of X-_N - X~_N against the level", "levels": LEVELS, "paths": PATHS,
           "variance": {}}
    for name, p in (("bf16_p8", fp.BF16), ("fp16_p11", fp.FP16), ("p17", fp.P17), ("fp32_p24", fp.FP32)):
        for kahan in (False, True):
            v = []
            for level in LEVELS:
                r = mlmc.level_sums(level, PATHS, GBM, rv_mode=mlmc.RV_CUBIC, precision=p, nested=False,
                                    kahan=kahan, seed=2, diag=True)
                v.append(mlmc.mean_var(r["sum"][3], r["sumsq"][3], PATHS)[1])
            out["variance"][name + ("_kahan" if kahan else "")] = v
    with open(os.path.join(HERE, "precision_sweep_oracle.json"), "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main()
