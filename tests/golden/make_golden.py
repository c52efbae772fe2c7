"""Writes the stored expected values under tests/golden/ from the CPU oracle alone.

Run from the repository root:  python tests/golden/make_golden.py
It imports nothing but ``oracle`` (and the standard library / NumPy / mpmath).

* dyadic_tables.json - the float64 master coefficient tables of the piecewise linear and
  piecewise cubic approximations of Phi^{-1} on 16 dyadic intervals of (0, 1/2]
  (Section 2.1, Figure 1, Lemmas 2.2 and 2.3; construction read as independent L2-optimal
  fits per interval), stored as exact hexadecimal floats; and the lower-half cell means of
  the piecewise-constant inverse CDF on 4096 equal cells of (0, 1) (a table-lookup
  approximate variable, Section 2.1), likewise.
"""

import json
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))

from oracle import tables  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    out = {}
    for key, degree in (("pwl16", 1), ("cubic16", 3)):
        tab = tables.compute_table(degree)
        out[key] = {
            "citation": "Section 2.1 (Figure 1; Lemma 2.2 piecewise linear, Lemma 2.3 "
                        "piecewise cubic): L2-optimal degree-%d fit of Phi^-1 in the local "
                        "coordinate t of each dyadic interval I_j = [2^-(j+1), 2^-j), "
                        "j=1..15, I_16 = (0, 2^-16)" % degree,
            "degree": degree,
            "coefficients": [[float(c).hex() for c in row] for row in tab],
        }
    bits = tables.PC_BITS
    out["pconst%d" % 2 ** bits] = {
        "citation": "Section 2.1 (approximate random variables by table lookup): the mean of "
                    "Phi^-1 over each of 2^%d equal cells of (0, 1), lower half" % bits,
        "bits": bits,
        "means": [float(m).hex() for m in tables.compute_pconst(bits)],
    }
    with open(os.path.join(HERE, "dyadic_tables.json"), "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main()
