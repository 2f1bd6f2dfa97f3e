"""CG-M (Algorithm 1 of the paper) in FP64, step by step.  Test infrastructure only.

The paper's Algorithm 1 solves (A + sigma I) x_sigma = b for all shifts from one Krylov
sequence (Section 2).  It is written here in the paper's order and notation:

* ``beta0`` is the step of the driving system; it is negative in this notation
  (r <- r + beta0 * Ap and x_sigma <- x_sigma - beta_sigma p_sigma), the convention of
  the multishift reference the paper builds on;
* ``alpha`` is the search-direction coefficient, p <- r + alpha p;
* ``zeta`` holds the collinearity factors, r_sigma = zeta_sigma r.

Three shifted constants are garbled as printed; they are replaced by the values that
follow from requiring r_sigma = zeta_sigma r for every iterate (derived by eliminating
p from the CG recurrences and matching the coefficients of r_{n+1}, r_n, r_{n-1}):

  zeta_{1s} = zeta_{0s} zeta_{-1s} beta_{-1}
              / (beta0 alpha (zeta_{-1s} - zeta_{0s}) + zeta_{-1s} beta_{-1} (1 - s beta0))
  beta_s    = beta0 zeta_{1s} / zeta_{0s}
  alpha_s   = alpha (zeta_{1s} / zeta_{0s})**2          (alpha already updated)
  p_s      <- zeta_{1s} r + alpha_s p_s                 (the new zeta, not the old one)

Further readings (the paper is silent or generic on these):

* the Krylov sequence is driven by the smallest shift sigma0 = min(sigma); the
  relative shifts s = sigma - sigma0 >= 0 enter the recurrences (the paper's A is the
  special case sigma0 = 0, available through ``drive``);
* the halting test is relative, |r| <= tol |b|, on the recursive residual of the
  driving system;
* a shift is frozen (no further update of x_s, p_s, zeta_s) once its recursive
  residual zeta_s^2 |r|^2 <= tol^2 |b|^2, which also keeps zeta from underflowing;
* a breakdown is reported when p^H (A + sigma0) p is not a positive finite number.
"""
from __future__ import annotations

import numpy as np


def _dot(u, v) -> complex:
    return complex(np.vdot(u, v))


def cg_m(apply_A, b, sigma, tol=1e-10, max_iter=10000, drive="min", freeze=True,
         observe=None):
    """Solve (A + sigma_k I) x_k = b for every shift with Algorithm 1 (corrected).

    Parameters
    ----------
    apply_A : callable ``apply_A(v, shift) -> (A + shift I) v`` in FP64.
    b       : complex right-hand side, shape (n,).
    sigma   : real shifts, any order, duplicates allowed.
    drive   : ``"min"`` (drive with the smallest shift) or a float sigma0.
    observe : optional ``observe(i, r=..., x=..., zeta=..., p=..., ps=...)`` called after
              every iteration with the state in sorted-shift order ``order``.

    Returns a dict with ``x`` (ns, n) in the caller's shift order, ``iters``, ``status``
    (``"ok"``, ``"notconv"`` or ``"breakdown"``), ``true_rel_res`` per shift,
    ``freeze_iter`` per shift (-1 if never frozen) and ``order`` (the sort of sigma).
    """
    b = np.asarray(b, dtype=np.complex128)
    sigma = np.asarray(sigma, dtype=np.float64).reshape(-1)
    ns, n = sigma.size, b.size
    order = np.argsort(sigma, kind="stable")
    sig = sigma[order]
    sigma0 = float(sig[0]) if drive == "min" else float(drive)
    s = sig - sigma0
    bnorm2 = _dot(b, b).real
    x_sorted = np.zeros((ns, n), dtype=np.complex128)
    freeze_iter = np.full(ns, -1, dtype=np.int64)
    result = dict(order=order, sigma0=sigma0)
    if bnorm2 == 0.0:
        result.update(x=np.zeros((ns, n), dtype=np.complex128), iters=0, status="ok",
                      true_rel_res=np.zeros(ns), freeze_iter=freeze_iter, R=0.0)
        return result
    eps2 = tol * tol * bnorm2

    # initialisation block of Algorithm 1
    alpha = 0.0
    beta0 = 1.0
    zeta_m1 = np.ones(ns)
    zeta_0 = np.ones(ns)
    r = b.copy()
    p = b.copy()
    p_s = np.tile(b, (ns, 1))
    x_s = x_sorted
    R1 = _dot(r, r).real
    i = 0
    active = np.ones(ns, dtype=bool)
    status = "notconv"

    while R1 > eps2 and i < max_iter:
        R0 = R1
        beta_m1 = beta0
        pbar = apply_A(p, sigma0)
        P = _dot(p, pbar).real
        if not (np.isfinite(P) and P > 0.0):
            status = "breakdown"
            break
        beta0 = -R0 / P
        r = r + beta0 * pbar
        act = np.nonzero(active)[0]
        zeta_1 = zeta_0.copy()
        denom = (beta0 * alpha * (zeta_m1[act] - zeta_0[act])
                 + zeta_m1[act] * beta_m1 * (1.0 - s[act] * beta0))
        zeta_1[act] = zeta_0[act] * zeta_m1[act] * beta_m1 / denom
        beta_s = beta0 * zeta_1[act] / zeta_0[act]
        R1 = _dot(r, r).real
        if not np.isfinite(R1):
            status = "breakdown"
            break
        alpha = R1 / R0
        alpha_s = alpha * (zeta_1[act] / zeta_0[act]) ** 2
        p = r + alpha * p
        x_s[act] -= beta_s[:, None] * p_s[act]
        p_s[act] = zeta_1[act, None] * r[None, :] + alpha_s[:, None] * p_s[act]
        zeta_m1[act] = zeta_0[act]
        zeta_0[act] = zeta_1[act]
        i += 1
        if freeze:
            done = active & (zeta_0 * zeta_0 * R1 <= eps2)
            freeze_iter[done] = i
            active &= ~done
        if observe is not None:
            observe(i, r=r, x=x_s, zeta=zeta_0, p=p, ps=p_s, order=order, sigma0=sigma0)
    if status != "breakdown":
        status = "ok" if R1 <= eps2 else "notconv"

    x = np.empty_like(x_s)
    x[order] = x_s
    fi = np.empty_like(freeze_iter)
    fi[order] = freeze_iter
    rel = np.empty(ns)
    bn = np.sqrt(bnorm2)
    for k in range(ns):
        res = b - apply_A(x[k], float(sigma[k]))
        rel[k] = np.linalg.norm(res) / bn
    result.update(x=x, iters=i, status=status, true_rel_res=rel, freeze_iter=fi, R=R1)
    return result
