"""Different right-hand sides per shift, (A + sigma_k I) x_k = b_k, through initial
guesses that give every shifted system the same residual.  Test infrastructure only.

The paper's discussion (Section 5, eq. linprobgen) notes that with x_k = 0 the residuals
b_k are independent, so the shifted systems would not share a Krylov space, and that a
judicious choice of initial guesses (after Osborn) makes all initial residuals equal, so
that one multishift solve finishes the family; it leaves the construction of the
guesses, which takes several products with A, to future GPU work.

Construction used here (written from that requirement).  Let s_0 < ... < s_{m-1} be the
shifts and b(s) = sum_j D_j w_j(s) the Newton interpolant of the right-hand sides
(D_j the divided differences b[s_0, ..., s_j], w_j(s) = prod_{l<j} (s - s_l)).  Look for
x(s) = sum_{j=0}^{m-2} Y_j w_j(s).  Since s w_j(s) = w_{j+1}(s) + s_j w_j(s),

    b(s) - (A + s) x(s) = [D_0 - (A + s_0) Y_0]
                          + sum_{j=1}^{m-2} [D_j - (A + s_j) Y_j - Y_{j-1}] w_j(s)
                          + [D_{m-1} - Y_{m-2}] w_{m-1}(s),

so Y_{m-2} = D_{m-1} and Y_{j-1} = D_j - (A + s_j) Y_j (j = m-2 .. 1) leave the residual
r_0 = D_0 - (A + s_0) Y_0 for every s: the guesses x0_k = x(s_k) satisfy
b_k - (A + s_k) x0_k = r_0 for all k, at the cost of m - 1 products with A.  A multishift
solve of (A + s_k) d_k = r_0 then gives x_k = x0_k + d_k.

Reading: nodes in ascending order of the shifts; the multishift stop is tightened to
tol min_k |b_k| / |r_0| so that every shift meets tol |b_k|; distinct shifts are required
(a repeated shift with different right-hand sides has no common residual).  The
interpolant is evaluated at the eigenvalues -lambda(A), far outside the interval of the
shifts, so |r_0| and the guesses grow with the spread of the shifts and with how much
the b_k differ; the solve stays exact in exact arithmetic but loses precision as that
growth approaches 1/eps.
"""
from __future__ import annotations

import numpy as np

from .cgm import cg_m


def common_residual_guesses(apply_A, B, sigma):
    """(x0 (m, n) in the caller's order, r0): b_k - (A + sigma_k) x0_k = r0 for every k."""
    B = np.asarray(B, dtype=np.complex128)
    sigma = np.asarray(sigma, dtype=np.float64).ravel()
    m = sigma.size
    if B.shape[0] != m:
        raise ValueError("one right-hand side per shift")
    order = np.argsort(sigma, kind="stable")
    s = sigma[order]
    if m > 1 and np.any(np.diff(s) == 0.0):
        raise ValueError("the shifts must be distinct")
    # divided differences, in place: D[j] = b[s_0, ..., s_j]
    D = B[order].copy()
    for level in range(1, m):
        for k in range(m - 1, level - 1, -1):
            D[k] = (D[k] - D[k - 1]) / (s[k] - s[k - level])
    # coefficients of x(s) in the Newton basis
    Y = [None] * max(m - 1, 0)
    if m >= 2:
        Y[m - 2] = D[m - 1].copy()
        for j in range(m - 2, 0, -1):
            Y[j - 1] = D[j] - apply_A(Y[j], float(s[j]))
        r0 = D[0] - apply_A(Y[0], float(s[0]))
    else:
        r0 = D[0].copy()
    x0 = np.zeros_like(B)
    for kk in range(m):
        acc = np.zeros(B.shape[1], dtype=np.complex128)
        w = 1.0
        for j in range(min(kk, m - 2) + 1):
            acc = acc + w * Y[j]
            w = w * (s[kk] - s[j])
        x0[order[kk]] = acc
    return x0, r0


def multi_rhs_solve(apply_A, B, sigma, tol=1e-10, max_iter=10000):
    """x_k = (A + sigma_k)^{-1} b_k for every k: the guesses above, then one CG-M on the
    common residual with the stop tightened to tol min_k |b_k| / |r0|.  Returns a dict with
    ``x``, ``x0``, ``r0``, the multishift ``iters`` and the FP64 ``true_rel_res``."""
    B = np.asarray(B, dtype=np.complex128)
    sigma = np.asarray(sigma, dtype=np.float64).ravel()
    x0, r0 = common_residual_guesses(apply_A, B, sigma)
    bn = np.linalg.norm(B, axis=1)
    rn = np.linalg.norm(r0)
    x = x0.copy()
    iters = 0
    if rn > 0.0:
        inner = cg_m(apply_A, r0, sigma, tol=tol * bn.min() / rn, max_iter=max_iter, verify=False)
        x = x0 + inner["x"]
        iters = inner["iters"]
    res = np.array([np.linalg.norm(B[k] - apply_A(x[k], float(sigma[k]))) for k in range(sigma.size)])
    return dict(x=x, x0=x0, r0=r0, iters=iters, true_rel_res=res / np.where(bn > 0, bn, 1.0))
