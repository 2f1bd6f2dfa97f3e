"""Multishift conjugate gradient (CG-M) in FP64.  Test infrastructure only.

What it computes (Section 2, eq. linprob and the discussion of shift invariance): the
solutions x_k = (A + sigma_k I)^{-1} b of a whole family of shifted systems from the one
Krylov sequence of a single "driving" system.

Derivation used here (restated from the mathematics, not from the printed algorithm,
whose shifted constants are garbled; Section 2, Algorithm 1 is the method being
restated).  Plain CG on the driving matrix B = A + sigma0 I with positive step sizes:

    q_n     = B d_n,             a_n = |r_n|^2 / d_n^H q_n
    r_{n+1} = r_n - a_n q_n,     c_n = |r_{n+1}|^2 / |r_n|^2
    d_{n+1} = r_{n+1} + c_n d_n

Eliminating d gives a three-term recurrence for the residuals alone.  The residual of
the shifted matrix B + s I (s = sigma_k - sigma0 >= 0) after n steps of CG lies in the
same Krylov space and, because both are the residual polynomial applied to b, is a
scalar multiple of r_n: r_n(s) = z_n(s) r_n.  Requiring that the same three-term
recurrence (with the shifted step a_n(s) and coefficient c_n(s)) holds for z_n(s) r_n
and matching the coefficients of r_{n+1}, r_n and r_{n-1} fixes

    z_{n+1} = z_n z_{n-1} a_{n-1} / ( a_n c_{n-1} (z_{n-1} - z_n)
                                      + z_{n-1} a_{n-1} (1 + s a_n) )
    a_n(s)  = a_n z_{n+1} / z_n
    c_n(s)  = c_n (z_{n+1} / z_n)^2

with z_{-1} = z_0 = 1, a_{-1} = 1, c_{-1} = 0.  Each shift then keeps its own iterate
and direction, x(s) += a_n(s) d(s) and d(s) <- z_{n+1} r_{n+1} + c_n(s) d(s).  The
driving system is the shift s = 0, for which z stays exactly 1.

Readings (the paper is silent or generic on these):

* the driving system is the smallest shift, sigma0 = min(sigma) (``drive`` may name
  another sigma0, e.g. 0 for the paper's unshifted A);
* halting is relative, |r_n| <= tol |b|, on the recursive residual of the driving system;
* a shift stops being advanced once its recursive residual z^2 |r|^2 <= tol^2 |b|^2,
  which also keeps z from underflowing;
* a breakdown is reported when d^H B d is not a positive finite number.
"""
from __future__ import annotations

import numpy as np


class _Shift:
    """State carried for one shifted system (in the sorted order of the shifts)."""

    def __init__(self, s, b):
        self.s = float(s)               # sigma_k - sigma0 >= 0
        self.x = np.zeros_like(b)       # iterate x(s)
        self.d = b.copy()               # direction d(s)
        self.z = 1.0                    # z_n(s):   r_n(s) = z_n(s) r_n
        self.z_old = 1.0                # z_{n-1}(s)
        self.live = True                # still advanced
        self.frozen_at = -1             # iteration at which it stopped, -1: never


def cg_m(apply_A, b, sigma, tol=1e-10, max_iter=10000, drive="min", freeze=True,
         observe=None, verify=True):
    """Solve (A + sigma_k I) x_k = b for every shift with one Krylov sequence.

    Parameters
    ----------
    apply_A : callable ``apply_A(v, shift) -> (A + shift I) v`` in FP64.
    b       : complex right-hand side, shape (n,).
    sigma   : real shifts, any order, duplicates allowed.
    drive   : ``"min"`` (drive with the smallest shift) or a float sigma0.
    observe : optional ``observe(i, r=..., x=..., zeta=..., p=..., ps=..., order=...,
              sigma0=...)`` called after every iteration with the state in sorted-shift
              order ``order`` (x, zeta and the directions ps stacked over the shifts).
    verify  : compute the true relative residual of every shift at the end (False: None).

    Returns a dict with ``x`` (ns, n) in the caller's shift order, ``iters``, ``status``
    (``"ok"``, ``"notconv"`` or ``"breakdown"``), ``true_rel_res`` per shift,
    ``freeze_iter`` per shift (-1 if never frozen) and ``order`` (the sort of sigma).
    """
    b = np.asarray(b, dtype=np.complex128)
    sigma = np.asarray(sigma, dtype=np.float64).reshape(-1)
    ns, n = sigma.size, b.size
    order = np.argsort(sigma, kind="stable")
    sigma0 = float(sigma[order[0]]) if drive == "min" else float(drive)
    shifts = [_Shift(sigma[k] - sigma0, b) for k in order]
    bb = float(np.vdot(b, b).real)
    result = dict(order=order, sigma0=sigma0)
    if bb == 0.0:
        result.update(x=np.zeros((ns, n), dtype=np.complex128), iters=0, status="ok",
                      true_rel_res=np.zeros(ns), freeze_iter=np.full(ns, -1, dtype=np.int64),
                      R=0.0)
        return result
    target = tol * tol * bb            # halting / freezing threshold on |r|^2

    r = b.copy()                       # driving residual
    d = b.copy()                       # driving direction
    rr = bb                            # |r_n|^2
    a_old, c_old = 1.0, 0.0            # a_{n-1}, c_{n-1}
    it = 0
    status = "notconv"
    while rr > target and it < max_iter:
        q = apply_A(d, sigma0)
        curv = float(np.vdot(d, q).real)
        if not (np.isfinite(curv) and curv > 0.0):
            status = "breakdown"
            break
        a = rr / curv
        # shifted steps from the collinearity of the residuals
        z_new = {}
        for j, sh in enumerate(shifts):
            if not sh.live:
                continue
            zn = sh.z * sh.z_old * a_old / (a * c_old * (sh.z_old - sh.z)
                                            + sh.z_old * a_old * (1.0 + sh.s * a))
            sh.x += (a * zn / sh.z) * sh.d
            z_new[j] = zn
        r = r - a * q
        rr_new = float(np.vdot(r, r).real)
        if not np.isfinite(rr_new):
            status = "breakdown"
            break
        c = rr_new / rr
        for j, zn in z_new.items():
            sh = shifts[j]
            ratio = zn / sh.z
            sh.d = zn * r + (c * ratio * ratio) * sh.d
            sh.z_old, sh.z = sh.z, zn
        d = r + c * d
        a_old, c_old, rr = a, c, rr_new
        it += 1
        if freeze:
            for sh in shifts:
                if sh.live and sh.z * sh.z * rr <= target:
                    sh.live = False
                    sh.frozen_at = it
        if observe is not None:
            observe(it, r=r, x=np.stack([sh.x for sh in shifts]),
                    zeta=np.array([sh.z for sh in shifts]), p=d,
                    ps=np.stack([sh.d for sh in shifts]), order=order, sigma0=sigma0)
    if status != "breakdown":
        status = "ok" if rr <= target else "notconv"

    x = np.empty((ns, n), dtype=np.complex128)
    frozen = np.empty(ns, dtype=np.int64)
    for j, k in enumerate(order):
        x[k] = shifts[j].x
        frozen[k] = shifts[j].frozen_at
    bn = np.sqrt(bb)
    rel = None
    if verify:
        rel = np.array([np.linalg.norm(b - apply_A(x[k], float(sigma[k]))) / bn
                        for k in range(ns)])
    result.update(x=x, iters=it, status=status, true_rel_res=rel, freeze_iter=frozen, R=rr)
    return result
