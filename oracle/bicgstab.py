"""BiCGStab and its multishift form BiCGStab-M in FP64.  Test infrastructure only.

The paper ships two shifted solvers, CG-M and BiCGStab-M (Section 1 and Section 3); it
prints only CG-M, so the shifted BiCGStab below is derived here from the mathematics,
for a general (non-Hermitian) sparse A and the family (A + sigma_k I) x_k = b (Section 2,
eq. linprob).

Plain BiCGStab on the driving matrix B = A + sigma0 I, shadow vector w = b:

    v_n = B p_n,            al_n = rho_n / w^H v_n,          s_n = r_n - al_n v_n
    t_n = B s_n,            om_n = t_n^H s_n / t_n^H t_n
    x_{n+1} = x_n + al_n p_n + om_n s_n,                     r_{n+1} = s_n - om_n t_n
    rho_{n+1} = w^H r_{n+1}, be_n = (rho_{n+1} / rho_n)(al_n / om_n)
    p_{n+1} = r_{n+1} + be_n (p_n - om_n v_n)

In polynomial form r_n = phi_n(B) pi_n(B) b and p_n = phi_n(B) theta_n(B) b, where
pi_n, theta_n are the residual and direction polynomials of BiCG,
    pi_{n+1} = pi_n - al_n z theta_n,   theta_{n+1} = pi_{n+1} + be_n theta_n,
and phi_n(z) = prod_{i<n} (1 - om_i z).

For B + s (s = sigma_k - sigma0) from the same Krylov space with the same shadow vector,
the BiCG residual is a multiple of the driving one, pi_n(s)(z + s) = pi_n(z) / pi_n(-s),
so z_n = 1 / pi_n(-s) obeys the same three-term recurrence as in CG-M:

    z_{n+1} = z_n z_{n-1} al_{n-1} / ( al_n be_{n-1} (z_{n-1} - z_n)
                                       + z_{n-1} al_{n-1} (1 + s al_n) )
    al_n(s) = al_n z_{n+1} / z_n,       be_n(s) = be_n (z_{n+1} / z_n)^2,

with z_{-1} = z_0 = 1, al_{-1} = 1, be_{-1} = 0 (complex in general).  Choosing the
shifted stabilising steps om_n(s) = om_n / (1 + s om_n) makes phi_n(s)(z + s) =
phi_n(z) / tau_n with tau_n = prod_{i<n} (1 + s om_i), so the shifted residual is the
driving one scaled: r_n(s) = (z_n / tau_n) r_n.  Likewise s_n(s) = (z_{n+1} / tau_n) s_n,
and B(s) p_n(s) never has to be formed: from al_n(s) (B + s) theta_n(s) = pi_n(s) -
pi_{n+1}(s),

    p_n(s) - om_n(s) (B + s) p_n(s) = p_n(s) - (om_n(s) / al_n(s)) (r_n(s) - s_n(s)),

so each shift keeps an iterate and a direction updated from r_n, s_n and r_{n+1}:

    x(s) += al_n(s) p(s) + om_n(s) (z_{n+1} / tau_n) s_n
    p(s)  = (z_{n+1} / tau_{n+1}) r_{n+1}
            + be_n(s) [ p(s) - (om_n(s) / al_n(s)) ((z_n / tau_n) r_n - (z_{n+1} / tau_n) s_n) ]

Readings: the driving system is the first shift in ascending order of sigma (any shift
would do); the shadow vector is b; every shift stops being advanced once its residual
|z_n / tau_n| |r_n| <= tol |b|, and the sequence halts when every shift has stopped; a
breakdown is reported when w^H v, t^H t or rho vanishes or 1 + s om_n = 0.
"""
from __future__ import annotations

import numpy as np


def bicgstab(apply_A, rhs, shift=0.0, tol=1e-10, max_iter=10000, record=False):
    """Textbook BiCGStab on (A + shift I) x = rhs from x = 0, shadow vector rhs."""
    rhs = np.asarray(rhs, dtype=np.complex128)
    x = np.zeros_like(rhs)
    r = rhs.copy()
    w = rhs.copy()
    p = r.copy()
    rho = np.vdot(w, r)
    ref = np.linalg.norm(rhs)
    history = [x.copy()] if record else None
    it = 0
    status = "notconv"
    while it < max_iter and np.linalg.norm(r) > tol * ref:
        v = apply_A(p, shift)
        wv = np.vdot(w, v)
        if wv == 0 or not np.isfinite(wv):
            status = "breakdown"
            break
        al = rho / wv
        s = r - al * v
        t = apply_A(s, shift)
        tt = np.vdot(t, t).real
        if tt == 0:
            x = x + al * p
            r = s
            it += 1
            if record:
                history.append(x.copy())
            break
        om = np.vdot(t, s) / tt
        x = x + al * p + om * s
        r = s - om * t
        rho_new = np.vdot(w, r)
        be = (rho_new / rho) * (al / om)
        p = r + be * (p - om * v)
        rho = rho_new
        it += 1
        if record:
            history.append(x.copy())
    if status != "breakdown":
        status = "ok" if np.linalg.norm(r) <= tol * ref else "notconv"
    out = dict(x=x, iters=it, status=status)
    if record:
        out["history"] = history
    return out


class _Shift:
    """State of one shifted system (sorted order)."""

    def __init__(self, s, b):
        self.s = float(s)
        self.x = np.zeros_like(b)
        self.p = b.copy()
        self.z = 1.0 + 0.0j        # z_n
        self.z_old = 1.0 + 0.0j    # z_{n-1}
        self.tau = 1.0 + 0.0j      # tau_n
        self.live = True
        self.frozen_at = -1


def bicgstab_m(apply_A, b, sigma, tol=1e-10, max_iter=10000, observe=None, verify=True):
    """Solve (A + sigma_k I) x_k = b for every shift with one BiCGStab sequence.

    Returns a dict: ``x`` (ns, n) in the caller's shift order, ``iters``, ``status``
    ("ok", "notconv", "breakdown"), ``freeze_iter`` (per shift) and, with ``verify``,
    ``true_rel_res`` (FP64 |b - (A + sigma_k) x_k| / |b|).  ``observe(n, r, shifts)``,
    if given, is called with the state after every iteration (for invariant checks).
    """
    b = np.asarray(b, dtype=np.complex128)
    sigma = np.asarray(sigma, dtype=np.float64).ravel()
    ns = sigma.size
    order = np.argsort(sigma, kind="stable")
    sigma0 = sigma[order[0]]
    shifts = [_Shift(sigma[k] - sigma0, b) for k in order]
    bnorm = np.linalg.norm(b)
    x_out = np.zeros((ns, b.size), dtype=np.complex128)
    if bnorm == 0.0:
        return dict(x=x_out, iters=0, status="ok", freeze_iter=np.zeros(ns, dtype=int),
                    true_rel_res=np.zeros(ns))
    w = b.copy()
    r = b.copy()
    p = b.copy()
    rho = np.vdot(w, r)
    al_prev, be_prev = 1.0 + 0.0j, 0.0 + 0.0j
    status = "notconv"
    it = 0
    while it < max_iter and any(sh.live for sh in shifts):
        v = apply_A(p, sigma0)
        wv = np.vdot(w, v)
        if wv == 0 or not np.isfinite(wv):
            status = "breakdown"
            break
        al = rho / wv
        s_vec = r - al * v
        # BiCG part of every shift: z_{n+1}, al_n(s)
        for sh in shifts:
            if not sh.live:
                continue
            den = al * be_prev * (sh.z_old - sh.z) + sh.z_old * al_prev * (1.0 + sh.s * al)
            sh.z_new = sh.z * sh.z_old * al_prev / den
            sh.al = al * sh.z_new / sh.z
        t = apply_A(s_vec, sigma0)
        tt = np.vdot(t, t).real
        if not (tt > 0) or not np.isfinite(tt):
            status = "breakdown"
            break
        om = np.vdot(t, s_vec) / tt
        r_new = s_vec - om * t
        rho_new = np.vdot(w, r_new)
        if rho_new == 0 or om == 0:
            # the sequence ends here: apply the last step and stop
            be = 0.0 + 0.0j
        else:
            be = (rho_new / rho) * (al / om)
        for sh in shifts:
            if not sh.live:
                continue
            g = 1.0 + sh.s * om
            if g == 0:
                status = "breakdown"
                break
            om_s = om / g
            tau_new = sh.tau * g
            sh.x = sh.x + sh.al * sh.p + om_s * (sh.z_new / sh.tau) * s_vec
            be_s = be * (sh.z_new / sh.z) ** 2
            back = (sh.z / sh.tau) * r - (sh.z_new / sh.tau) * s_vec
            sh.p = (sh.z_new / tau_new) * r_new + be_s * (sh.p - (om_s / sh.al) * back)
            sh.z_old, sh.z, sh.tau = sh.z, sh.z_new, tau_new
        if status == "breakdown":
            break
        p = r_new + be * (p - om * v)
        r, rho = r_new, rho_new
        al_prev, be_prev = al, be
        it += 1
        rn = np.linalg.norm(r)
        for sh in shifts:
            if sh.live and abs(sh.z / sh.tau) * rn <= tol * bnorm:
                sh.live = False
                sh.frozen_at = it
        if observe is not None:
            observe(it, r, shifts)
        if rho == 0 or om == 0:
            break
    if status != "breakdown":
        status = "ok" if not any(sh.live for sh in shifts) else "notconv"
    freeze = np.full(ns, -1, dtype=int)
    for j, k in enumerate(order):
        x_out[k] = shifts[j].x
        freeze[k] = shifts[j].frozen_at
    out = dict(x=x_out, iters=it, status=status, freeze_iter=freeze)
    if verify:
        out["true_rel_res"] = np.array(
            [np.linalg.norm(b - apply_A(x_out[k], sigma[k])) for k in range(ns)]) / bnorm
    return out
