"""CPU FP64 oracle for sketch-preconditioned Tikhonov least squares.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) may import, call, link or execute anything in this package;
only the tests, the smoke check and the benchmark's CPU-baseline leg do.  It
shares no code with the GPU path: it never touches the GPU, the binding or
the C library, and it receives its inputs from the seeded generators in
``workloads``.

What it computes (each function cites the passage it follows):

* ``tikhonov.solve``  x_lam = argmin ||Ax-b||^2 + lam ||x||^2 for every lam
  (eq. regLLS), by the direct Householder-QR route the paper names as the
  classical alternative (Section 1.2): QR of [A; sqrt(lam) I] with right-hand
  side [b; 0] (eq. regLLSover) when m >= n, and the minimum-norm solution of
  [A sqrt(lam) I] z = b (eq. regLLSunder) when m < n.
* ``tikhonov.statistical_dimension`` (Definition 1) and ``sd_hat`` (the
  estimate from the sketch's singular values, Section 3.1.2).
* ``tikhonov.chol_precond`` / ``bp2_precond`` (the QR route of Section 4.1)
  / ``lowrank_factors`` / ``lowrank_rinv``: the
  preconditioners of Algorithms 1-3 written out densely for small checks;
  ``lowrank_truncation`` the rank s_i each lambda keeps (Algorithm 3).
* ``tikhonov.lsqr_iteration_bound`` and the Lemma 2.1 / Theorem 3.2 bounds.
* ``tikhonov.lcurve_norms`` / ``lcurve_curvature`` / ``lcurve_corner``: the
  L-curve of Section 4.3 and its maximum-curvature corner.
* ``tikhonov.certify``: an a-posteriori bound on the forward error of a
  candidate solution that holds at any size; ``certify_planted`` sharpens it
  with the generator's planted factors (used at full size, where the direct
  solve takes minutes).  Both accumulate the gradient in extended precision
  (``grad_ld.c``, plain C, built by ``native.build_native``).

Parity status: every function above is pinned by tests in
tests/test_oracle_pins.py against closed forms, exact rational arithmetic,
a LAPACK cross-check, an independent LSQR (scipy's, for the iteration bound)
or the paper's own identities (the wide-problem factors against the mirror
of the BP2 equivalence, the underdetermined condition lemma of Section 2.2
and the theorem of Section 3.3.2).
"""

from .tikhonov import (  # noqa: F401
    solve,
    solve_over,
    solve_under,
    statistical_dimension,
    sd_hat,
    lowrank_S,
    lowrank_factors,
    lowrank_rinv,
    lowrank_truncation,
    chol_precond,
    chol_precond_under,
    bp2_precond,
    lsqr_iteration_bound,
    lemma21_bound,
    thm32_bound,
    thm32_eps,
    rel_err,
    certify,
    certify_planted,
    lcurve_norms,
    lcurve_curvature,
    lcurve_corner,
)
