"""Pins of the FP64 oracle against what the mathematics fixes (no GPU).

Each test checks the oracle against something other than itself: a dense LAPACK solve,
the free-field Fourier closed form, the pure-gauge closed form, the collinearity
invariant r_k = zeta_k r, the textbook CG iterates of each shifted system, the
closed-form first step, and the halting / breakdown special cases.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W


def _problem(name="c0"):
    p = W.make_config(name)
    p["apply"] = O.shifted_apply(p["kind"], p["rowptr"], p["col"], p["vals"], p["n"])
    return p


@pytest.fixture(scope="module")
def c0():
    return _problem("c0")


def _cond(kind, rowptr, col, vals, n, sigma):
    m = O.dense_from_csr(rowptr, col, vals, n)
    a = m.conj().T @ m if kind == "mhm" else m
    ev = np.linalg.eigvalsh(a)
    return (ev.max() + sigma) / (ev.min() + sigma)


def test_c0_against_dense_solve(c0):
    res = O.cg_m(c0["apply"], c0["b"], c0["sigma"], tol=1e-10)
    assert res["status"] == "ok"
    assert np.all(res["true_rel_res"] <= 1e-10)
    xd = O.dense_solve("mhm", c0["rowptr"], c0["col"], c0["vals"], c0["n"], c0["b"], c0["sigma"])
    kappa = _cond("mhm", c0["rowptr"], c0["col"], c0["vals"], c0["n"], c0["sigma"])
    err = np.linalg.norm(res["x"] - xd, axis=1) / np.linalg.norm(xd, axis=1)
    assert np.all(err <= kappa * res["true_rel_res"] * 1.01 + 1e-13)
    assert np.all(err <= 1e-9)


def test_non_normal_matrix_distinguishes_mhm_from_mmh():
    rowptr, col, vals = W.random_sparse_csr(120, 5, 17, diag=4.0)
    b = W.gaussian_rhs(120, 18)
    sigma = np.array([0.3, 0.01, 2.0, 0.05])
    ap = O.shifted_apply("mhm", rowptr, col, vals, 120)
    res = O.cg_m(ap, b, sigma, tol=1e-12)
    xd = O.dense_solve("mhm", rowptr, col, vals, 120, b, sigma)
    m = O.dense_from_csr(rowptr, col, vals, 120)
    wrong = np.linalg.solve(m @ m.conj().T + 0.3 * np.eye(120), b)
    assert np.linalg.norm(res["x"] - xd) / np.linalg.norm(xd) < 1e-9
    assert np.linalg.norm(res["x"][0] - wrong) / np.linalg.norm(wrong) > 1e-3


def test_herm_kind_against_dense_solve():
    rowptr, col, vals = W.laplacian7_csr((5, 4, 6), 3)
    n = 120
    b = W.gaussian_rhs(n, 4)
    sigma = W.logspace_shifts(1e-4, 1.0, 10)
    res = O.cg_m(O.shifted_apply("herm", rowptr, col, vals, n), b, sigma, tol=1e-12)
    xd = O.dense_solve("herm", rowptr, col, vals, n, b, sigma)
    assert res["status"] == "ok"
    assert np.linalg.norm(res["x"] - xd) / np.linalg.norm(xd) < 1e-10


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 4, 8)])
def test_free_field_closed_form(dims):
    mass = 0.1
    rowptr, col, vals = W.staggered_csr(W.free_links(dims), dims, mass)
    n = 3 * W.lattice_volume(dims)
    b = W.gaussian_rhs(n, 40)
    sigma = W.logspace_shifts(1e-4, 1.0, 6)
    res = O.cg_m(O.shifted_apply("mhm", rowptr, col, vals, n), b, sigma, tol=1e-11)
    xf = O.free_field_solve(dims, mass, b, sigma)
    kappa = (4.0 + mass ** 2 + sigma) / (mass ** 2 + sigma)
    err = np.linalg.norm(res["x"] - xf, axis=1) / np.linalg.norm(xf, axis=1)
    assert np.all(err <= kappa * 1e-11)


def test_free_field_closed_form_is_the_inverse():
    # the Fourier closed form itself, checked against a dense solve
    dims = (4, 4, 4, 4)
    rowptr, col, vals = W.staggered_csr(W.free_links(dims), dims, 0.2)
    b = W.gaussian_rhs(768, 41)
    sigma = [0.0, 0.5]
    xf = O.free_field_solve(dims, 0.2, b, sigma)
    xd = O.dense_solve("mhm", rowptr, col, vals, 768, b, sigma)
    assert np.abs(xf - xd).max() < 1e-12 * np.abs(xd).max()


def test_pure_gauge_closed_form():
    dims = (4, 4, 4, 4)
    links, g = W.pure_gauge_links(dims, 42)
    rowptr, col, vals = W.staggered_csr(links, dims, 0.1)
    b = W.gaussian_rhs(768, 43)
    sigma = W.logspace_shifts(1e-4, 1.0, 5)
    res = O.cg_m(O.shifted_apply("mhm", rowptr, col, vals, 768), b, sigma, tol=1e-11)
    xp = O.pure_gauge_solve(dims, 0.1, g, b, sigma)
    kappa = (4.01 + sigma) / (0.01 + sigma)
    err = np.linalg.norm(res["x"] - xp, axis=1) / np.linalg.norm(xp, axis=1)
    assert np.all(err <= kappa * 1e-11)


def test_collinearity_every_iteration(c0):
    """b - (A + sigma_k) X_k^(n) = zeta_k^(n) r^(n) for every n (no freezing)."""
    b, ap = c0["b"], c0["apply"]
    bn = np.linalg.norm(b)
    worst = [0.0]

    def observe(i, r, x, zeta, order, sigma0, **_):
        if i > 100:
            return
        sig = c0["sigma"][order]
        for k in range(len(sig)):
            res_k = b - ap(x[k], float(sig[k]))
            worst[0] = max(worst[0], np.linalg.norm(res_k - zeta[k] * r) / bn)

    O.cg_m(ap, b, c0["sigma"], tol=1e-10, freeze=False, observe=observe, max_iter=100)
    assert worst[0] < 1e-12


def test_single_shift_is_textbook_cg(c0):
    """Ns = 1: zeta = 1 and the iterates are those of plain CG on A + sigma."""
    b, ap = c0["b"], c0["apply"]
    hist = []
    O.cg_m(ap, b, [0.05], tol=1e-10, observe=lambda i, x, zeta, **_: hist.append(
        (x[0].copy(), zeta[0])), max_iter=40)
    ref = O.cg(ap, b, shift=0.05, tol=0.0, max_iter=40, record=True)["history"]
    for n, (xn, zn) in enumerate(hist, start=1):
        assert zn == 1.0
        assert np.linalg.norm(xn - ref[n]) <= 1e-13 * np.linalg.norm(ref[n])


@pytest.mark.parametrize("drive", ["min", 0.0])
def test_iterates_equal_per_shift_cg(c0, drive):
    """X_k^(n) equals n steps of plain CG on (A + sigma_k) from 0, for n <= 20."""
    b, ap, sigma = c0["b"], c0["apply"], c0["sigma"]
    hist = []
    O.cg_m(ap, b, sigma, tol=0.0, freeze=False, drive=drive, max_iter=20,
           observe=lambda i, x, order, **_: hist.append((x.copy(), order)))
    for k, sk in enumerate(sigma):
        ref = O.cg(ap, b, shift=float(sk), tol=0.0, max_iter=20, record=True)["history"]
        for n, (xs, order) in enumerate(hist, start=1):
            kk = int(np.nonzero(order == k)[0][0])
            assert np.linalg.norm(xs[kk] - ref[n]) <= 1e-9 * np.linalg.norm(ref[n])


def test_first_step_closed_form(c0):
    b, ap, sigma = c0["b"], c0["apply"], c0["sigma"]
    snap = {}

    def observe(i, x, zeta, order, sigma0, **_):
        if i == 1:
            snap.update(x=x.copy(), zeta=zeta.copy(), order=order, sigma0=sigma0)

    O.cg_m(ap, b, sigma, tol=0.0, max_iter=1, observe=observe)
    bb = np.vdot(b, b).real
    a0 = bb / np.vdot(b, ap(b, snap["sigma0"])).real
    for kk, k in enumerate(snap["order"]):
        s = sigma[k] - snap["sigma0"]
        assert snap["zeta"][kk] == pytest.approx(1.0 / (1.0 + s * a0), rel=1e-15)
        step = bb / np.vdot(b, ap(b, float(sigma[k]))).real
        assert np.abs(snap["x"][kk] - step * b).max() <= 1e-15 * np.abs(step * b).max()


def test_zeta_monotone(c0):
    b, ap, sigma = c0["b"], c0["apply"], c0["sigma"]
    zs = [np.ones(sigma.size)]
    O.cg_m(ap, b, sigma, tol=1e-10, freeze=True,
           observe=lambda i, zeta, **_: zs.append(zeta.copy()))
    zs = np.array(zs)
    assert np.all(zs > 0.0)
    assert np.all(np.diff(zs, axis=0) <= 0.0)
    assert np.all(zs <= 1.0)


def test_iteration_count_matches_driving_cg(c0):
    res = O.cg_m(c0["apply"], c0["b"], c0["sigma"], tol=1e-10)
    ref = O.cg(c0["apply"], c0["b"], shift=float(c0["sigma"].min()), tol=1e-10)
    assert abs(res["iters"] - ref["iters"]) <= 2


def test_caller_order_and_duplicates(c0):
    b, ap = c0["b"], c0["apply"]
    sigma = np.array([0.5, 1e-3, 0.5, 0.02])
    res = O.cg_m(ap, b, sigma, tol=1e-11)
    xd = O.dense_solve("mhm", c0["rowptr"], c0["col"], c0["vals"], c0["n"], b, sigma)
    assert np.linalg.norm(res["x"] - xd) / np.linalg.norm(xd) < 1e-9
    assert np.array_equal(res["x"][0], res["x"][2])


def test_zero_rhs(c0):
    res = O.cg_m(c0["apply"], np.zeros(c0["n"], complex), c0["sigma"])
    assert res["iters"] == 0 and res["status"] == "ok" and not np.any(res["x"])


def test_iteration_limit(c0):
    res = O.cg_m(c0["apply"], c0["b"], c0["sigma"], max_iter=1)
    assert res["status"] == "notconv" and res["iters"] == 1


def test_indefinite_shift_breaks_down(c0):
    res = O.cg_m(c0["apply"], c0["b"], [-50.0, 1.0], tol=1e-10)
    assert res["status"] == "breakdown"


def test_freezing_keeps_every_shift_converged(c0):
    res = O.cg_m(c0["apply"], c0["b"], c0["sigma"], tol=1e-10, freeze=True)
    fi = res["freeze_iter"]
    # larger shifts converge (and freeze) no later than smaller ones
    order = np.argsort(c0["sigma"])
    assert np.all(np.diff(fi[order]) <= 0)
    assert np.all(res["true_rel_res"] <= 1e-10)
