"""CPU oracle for the MLMC level-correction estimator of Euler-Maruyama SDE paths.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously-correct restatement,
in float64 NumPy (with per-operation float32 / float16 emulation where the method runs in
a lower precision), of what the GPU library computes.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may import it.
The product path (``paper_2012_09739_amd``) never imports, calls or links anything here,
and nothing here imports the product.  The two share no code: the oracle has its own
Philox, its own inverse normal CDF (SciPy's ``ndtri``), its own approximation tables
(mpmath quadrature) and its own Euler-Maruyama loop.

Modules (each function cites the passage of the paper it restates):

* ``philox``   - Philox4x32-10 counter-based uniforms (the paper leaves the generator open;
                 the counter layout is the build's reading, see ``philox.word``).
* ``tables``   - L2-optimal piecewise-polynomial fits of the inverse Gaussian CDF on 16
                 dyadic intervals of (0, 1/2] (Section 2.1, Figure 1, Lemmas 2.2 and 2.3).
* ``icdf``     - exact Z = Phi^{-1}(U) and approximate Z~ = Phi~^{-1}(U) from the same
                 uniform (Section 3, the coupling of exact and approximate variables).
* ``fp``       - the precision model: IEEE round-to-nearest-even in binary64/32/16
                 (Section 2.2, the standard rounding model).
* ``mlmc``     - coupled fine/coarse Euler-Maruyama paths in finite precision, optional
                 Kahan-compensated state updates, payoffs, the two-way and four-way
                 differences and their sums (Sections 2.2, 2.3 and 3).
* ``mlp``      - the 1-16-16-1 tanh surrogate for the inverse CDF: float64 forward pass,
                 analytic back-propagation and the loss (a learned approximate random
                 variable; the paper's Section 2.1 allows any approximation meeting
                 Assumption 2.1 -- this one is mirrored, hence exactly zero mean).

Parity status of each function is recorded in its docstring; every function is pinned
by a ``-m "not gpu"`` test against something other than itself (closed forms, library
routines, brute force, mpmath), except where a docstring says "parity unpinned".
"""

from . import fp, philox, tables, icdf, mlp, mlmc  # noqa: F401
