"""FP64 CPU oracle for SubApSnap (Jones & Nakatsukasa, arXiv 2510.04825).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, deliberately
unoptimised NumPy/SciPy implementation of what the GPU library computes.  It
exists to check the GPU path; only the test suite, the package smoke check and
the benchmark's CPU-baseline leg may import it.  It shares no code with the
GPU library (no kernels, headers, tables or helpers) and imports nothing from
it; its inputs come from ``subap_inputs`` (random draws only) or from the
paper.

Layout
------
families  -- the parameter-dependent systems A(p) x = b(p) (eq. (1.1)):
             finite-difference diffusion in 2-D/3-D, Gaussian-kernel ridge
             regression (eqs. (6.3)-(6.4)), the shifted tridiagonal example
             (eq. (5.7)) and the identity family (DEIM, eq. (3.5)).
offline   -- Algorithm 3.1 steps 1-3: snapshot solves, orthonormalisation
             (Section 3.1, "Postprocessing the snapshot matrix"), and row
             selection by column-pivoted QR on (A(p) X)^T (Section 5.3).
online    -- Algorithm 3.1 step 4: rows of A(p*), S A(p*) X, the s x r least
             squares problem (eq. (3.3)), the lift X c, residual measures and
             ApSnap (eq. (3.1)) as the full-sampling reference.
mlp       -- FP64 forward/backward/Adam for the learned p -> y surrogate.

Parity status of each function is stated in its docstring; every function
here is pinned by a test in ``tests/test_oracle_*.py`` against a closed form,
a library routine on a special case, or a fact the paper states.
"""
from . import families, offline, online, mlp  # noqa: F401
