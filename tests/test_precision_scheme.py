"""Why the mixed solve switches precision instead of running complex64 throughout (no GPU).

A numpy emulation of the multishift CG sequence (paper: Section 2, Algorithm 1) under
three precision schemes, each with FP64 scalars, FP64 reductions, complex128 x_k and a
FP64 true-residual replacement of the driving residual every 50 complex64 iterations:

  A  the library's: FP64 until |r| <= 3e-5 |b|, then complex64 operator, r, p, t and
     shift directions p_k;
  B  complex64 operator, r, p, t and p_k from the first iteration;
  C  complex64 operator, r, p, t from the first iteration, p_k kept in complex128.

What fixes each shifted solution is the consistency of x_k with the implicit residual
zeta_k r: rounding injected while |r| ~ |b| (early iterations, zeta_k ~ 1) leaves a gap
between the true and the implicit residual that no replacement of the driving residual
removes.  Only scheme A keeps every shift within a few tol of tol; B and C would need most
shifts refined from 1e-7..1e-4 (about as much work again as the sequence itself).
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W


def _emulate(scheme, dims=(4, 4, 4, 4), mass=0.02, tol=1e-10, sw=3e-5, ru_every=50):
    links = W.random_su3_links(dims, 11)
    rp, col, vals = W.staggered_csr(links, dims, mass)
    n = 3 * W.lattice_volume(dims)
    M = sp.csr_matrix((vals, col, rp), shape=(n, n))
    MH = M.conj().T.tocsr()
    M32, MH32 = M.astype(np.complex64), MH.astype(np.complex64)
    b = W.gaussian_rhs(n, 3)
    sig = W.logspace_shifts(1e-6, 10.0, 16)
    s0 = sig[0]
    s = sig - s0
    ns = sig.size

    def a64(v, sh=s0):
        return MH @ (M @ v) + sh * v

    def a32(v):
        v32 = v.astype(np.complex64)
        return ((MH32 @ (M32 @ v32)) + np.complex64(s0) * v32).astype(complex)

    def low(v):
        return v.astype(np.complex64).astype(complex)

    x = np.zeros((ns, n), complex)
    pk = np.tile(b, (ns, 1)).astype(complex)
    r, p = b.copy(), b.copy()
    R = B2 = float(np.vdot(b, b).real)
    z, zm, ap, bc = np.ones(ns), np.ones(ns), 1.0, 0.0
    active = np.ones(ns, bool)
    fp64 = scheme == "A"
    if not fp64:
        r, p = low(r), low(p)
        if scheme == "B":
            pk = low(pk)
    since = 0
    for _ in range(20000):
        w = a64(p) if fp64 else a32(p)
        a = R / float(np.vdot(p, w).real)
        zn = np.where(active, z * zm * ap / (a * bc * (zm - z) + zm * ap * (1 + s * a)), z)
        ak = a * zn / z
        for k in np.flatnonzero(active):
            x[k] += ak[k] * pk[k]
        r = r - a * w
        if not fp64:
            r = low(r)
            since += 1
            if since % ru_every == 0:
                r = low(b - a64(x[0]))
        Rn = float(np.vdot(r, r).real)
        bn = Rn / R
        bk = bn * (zn / z) ** 2
        for k in np.flatnonzero(active):
            pk[k] = zn[k] * r + bk[k] * pk[k]
            if not fp64 and scheme != "C":
                pk[k] = low(pk[k])
        p = r + bn * p
        if not fp64:
            p = low(p)
        zm, z, ap, bc, R = z, zn, a, bn, Rn
        active &= z ** 2 * R > (0.7 * tol) ** 2 * B2
        active[0] = True
        if fp64 and scheme == "A" and R <= sw ** 2 * B2:
            fp64 = False
            r, p, pk = low(r), low(p), low(pk)
            since = 0
        if R <= (0.7 * tol) ** 2 * B2:
            break
    return np.array([np.linalg.norm(b - a64(x[k], sig[k])) for k in range(ns)]) / np.sqrt(B2)


@pytest.fixture(scope="module")
def gaps():
    return {sc: _emulate(sc) for sc in ("A", "B", "C")}


def test_switching_scheme_keeps_every_shift_near_tol(gaps):
    res = gaps["A"]
    assert res[0] <= 1e-10
    assert res.max() <= 1e-8          # measured 1.3e-9: a few shifts refined, briefly


def test_complex64_throughout_leaves_large_gaps(gaps):
    # complex64 shift directions from the start: gaps of order 1e-5 |b|
    assert gaps["B"][0] <= 1e-10       # the driving shift itself is fine
    assert gaps["B"][1:].max() >= 1e-6
    assert np.sum(gaps["B"] > 1e-10) >= 12


def test_complex128_directions_alone_do_not_close_the_gap(gaps):
    # FP64 p_k with a complex64 driving sequence: the driving residual's own rounding,
    # injected while zeta_k ~ 1, still leaves gaps far above tol
    assert gaps["C"][1:].max() >= 1e-8
    assert gaps["C"][1:].max() >= 10 * gaps["A"][1:].max()
