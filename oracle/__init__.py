"""FP64 CPU oracle for the multishift conjugate-gradient solve.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU library never
calls it, shares no code with it, and fails loudly when its compiled extension is
missing instead of falling back to anything here.

Contents (each function cites the passage of the paper it follows):

* :mod:`oracle.cgm`      -- Algorithm 1 (CG-M) step by step, with the printed errata
                            corrected, plus the true per-shift residuals.
* :mod:`oracle.cg`       -- textbook unshifted CG (the paper's comparator, Section 4).
* :mod:`oracle.bicgstab` -- textbook BiCGStab and the multishift BiCGStab-M (the
                            paper's second shifted solver, Sections 1 and 3) for
                            non-Hermitian A, derived from the BiCG polynomials.
* :mod:`oracle.osborn`   -- a different right-hand side per shift (Section 5, eq.
                            linprobgen): initial guesses that leave every shifted system
                            the same residual, then one CG-M.
* :mod:`oracle.direct`   -- the plain definition x_k = (A + sigma_k I)^{-1} b: dense
                            solve, the free-field Fourier closed form and the pure-gauge
                            closed form.
* :mod:`oracle.gradient` -- reference gradients of L = sum_k Re(g_k^H x_k): dense
                            autograd, the closed form for g_k = c_k b, and central
                            finite differences of a second-order functional (per
                            stored entry, or along one direction of all of them).
"""
from .operators import csr_matrix_of, shifted_apply, adjoint_csr
from .cgm import cg_m
from .cg import cg
from .bicgstab import bicgstab, bicgstab_m
from .osborn import common_residual_guesses, multi_rhs_solve
from .direct import dense_from_csr, dense_solve, free_field_solve, pure_gauge_solve
from .gradient import (
    dense_reference_gradient,
    closed_form_gradient,
    adjoint_gradient,
    fd_gradient,
    fd_directional,
    second_order_loss,
)

__all__ = [
    "csr_matrix_of",
    "shifted_apply",
    "adjoint_csr",
    "cg_m",
    "cg",
    "bicgstab",
    "bicgstab_m",
    "common_residual_guesses",
    "multi_rhs_solve",
    "dense_from_csr",
    "dense_solve",
    "free_field_solve",
    "pure_gauge_solve",
    "dense_reference_gradient",
    "closed_form_gradient",
    "adjoint_gradient",
    "fd_gradient",
    "fd_directional",
    "second_order_loss",
]
