"""Textbook (Hestenes-Stiefel) conjugate gradient in FP64.  Test infrastructure only.

This is the unshifted CG the paper compares against (Section 4, Table 1), applied to a
single shifted system (A + shift I) x = rhs.  It is also the n-step reference for the
multishift iterates: in exact arithmetic the n-th CG-M iterate of shift k equals the
n-th iterate of this method on A + sigma_k from x = 0 (Section 2: the Krylov spaces of
A and A + sigma I coincide, and the iterate is a polynomial in A applied to b).
"""
from __future__ import annotations

import numpy as np


def cg(apply_A, rhs, shift=0.0, x0=None, tol=1e-10, max_iter=10000, record=False,
       tol_ref=None):
    """Plain CG on (A + shift I) x = rhs.

    Stops when |r| <= tol * tol_ref (``tol_ref`` defaults to |rhs|) or after
    ``max_iter`` iterations.  Returns a dict with ``x``, ``iters``, ``status`` and, when
    ``record`` is set, the list ``history`` of iterates x^(0), x^(1), ...
    """
    rhs = np.asarray(rhs, dtype=np.complex128)
    x = np.zeros_like(rhs) if x0 is None else np.array(x0, dtype=np.complex128)
    r = rhs - apply_A(x, shift) if x0 is not None else rhs.copy()
    ref = np.linalg.norm(rhs) if tol_ref is None else float(tol_ref)
    p = r.copy()
    rr = np.vdot(r, r).real
    history = [x.copy()] if record else None
    it = 0
    status = "notconv"
    while it < max_iter and np.sqrt(rr) > tol * ref:
        q = apply_A(p, shift)
        pq = np.vdot(p, q).real
        if not (np.isfinite(pq) and pq > 0.0):
            status = "breakdown"
            break
        step = rr / pq
        x = x + step * p
        r = r - step * q
        rr_new = np.vdot(r, r).real
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
        if record:
            history.append(x.copy())
    if status != "breakdown":
        status = "ok" if np.sqrt(rr) <= tol * ref else "notconv"
    out = dict(x=x, iters=it, status=status, rnorm=np.sqrt(rr))
    if record:
        out["history"] = history
    return out
