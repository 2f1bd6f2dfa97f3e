"""Pins of the oracle's reference gradients (no GPU).

Three routes must agree: dense autograd through LAPACK solves, the closed form built
from oracle solutions, and central finite differences of the second-order functional.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_torch_convention_on_dense_fd():
    """grad = dL/dRe + i dL/dIm, checked by plain central differences of dense solves."""
    n = 12
    rowptr, col, vals = W.random_sparse_csr(n, 3, 5, diag=3.0)
    b = W.gaussian_rhs(n, 6)
    sigma = np.array([0.1, 0.7])
    g = W.gaussian_rhs(n, 7, 2)

    def loss(v, bb):
        x = O.dense_solve("mhm", rowptr, col, v, n, bb, sigma)
        return sum(np.real(np.vdot(g[k], x[k])) for k in range(2))

    gv, gb = O.dense_reference_gradient("mhm", rowptr, col, vals, n, b, sigma, g)
    h = 1e-6
    for e in (0, 5, len(vals) - 1):
        fd = 0j
        for unit in (1.0, 1j):
            vp, vm = vals.copy(), vals.copy()
            vp[e] += unit * h
            vm[e] -= unit * h
            fd += unit * (loss(vp, b) - loss(vm, b)) / (2 * h)
        assert abs(fd - gv[e]) <= 1e-7 * max(1.0, abs(gv[e]))
    for i in (0, 7):
        fd = 0j
        for unit in (1.0, 1j):
            bp, bm = b.copy(), b.copy()
            bp[i] += unit * h
            bm[i] -= unit * h
            fd += unit * (loss(vals, bp) - loss(vals, bm)) / (2 * h)
        assert abs(fd - gb[i]) <= 1e-7 * max(1.0, abs(gb[i]))


@pytest.fixture(scope="module")
def c3_4():
    p = W.make_config("c3_4")
    p["apply"] = O.shifted_apply("mhm", p["rowptr"], p["col"], p["vals"], p["n"])
    p["sol"] = O.cg_m(p["apply"], p["b"], p["sigma"], tol=1e-14, max_iter=100000)
    return p


def test_closed_form_matches_dense_autograd(c3_4):
    p = c3_4
    g = p["c"][:, None] * p["b"][None, :]
    gv_d, gb_d = O.dense_reference_gradient("mhm", p["rowptr"], p["col"], p["vals"], p["n"],
                                            p["b"], p["sigma"], g)
    gv_c, gb_c = O.closed_form_gradient("mhm", p["rowptr"], p["col"], p["vals"], p["n"],
                                        p["sol"]["x"], p["c"])
    assert _rel(gv_c, gv_d) < 1e-10
    assert _rel(gb_c, gb_d) < 1e-10


def test_general_adjoint_matches_dense_autograd(c3_4):
    p = c3_4
    g = W.gaussian_rhs(p["n"], 77, p["sigma"].size)
    y = np.stack([O.cg(p["apply"], g[k], shift=float(s), tol=1e-14, max_iter=100000)["x"]
                  for k, s in enumerate(p["sigma"])])
    gv_a, gb_a = O.adjoint_gradient("mhm", p["rowptr"], p["col"], p["vals"], p["n"],
                                    p["sol"]["x"], y)
    gv_d, gb_d = O.dense_reference_gradient("mhm", p["rowptr"], p["col"], p["vals"], p["n"],
                                            p["b"], p["sigma"], g)
    assert _rel(gv_a, gv_d) < 1e-10
    assert _rel(gb_a, gb_d) < 1e-10


def test_herm_adjoint_matches_dense_autograd():
    rowptr, col, vals = W.laplacian7_csr((4, 3, 5), 8)
    n = 60
    b = W.gaussian_rhs(n, 9)
    sigma = np.array([1e-3, 0.2, 1.0])
    g = W.gaussian_rhs(n, 10, 3)
    x = O.dense_solve("herm", rowptr, col, vals, n, b, sigma)
    y = np.stack([O.dense_solve("herm", rowptr, col, vals, n, g[k], [s])[0]
                  for k, s in enumerate(sigma)])
    gv_a, gb_a = O.adjoint_gradient("herm", rowptr, col, vals, n, x, y)
    gv_d, gb_d = O.dense_reference_gradient("herm", rowptr, col, vals, n, b, sigma, g)
    assert _rel(gv_a, gv_d) < 1e-12
    assert _rel(gb_a, gb_d) < 1e-12


def test_second_order_loss_is_exact_at_solution(c3_4):
    p = c3_4
    lt = O.second_order_loss("mhm", p["rowptr"], p["col"], p["vals"], p["n"], p["b"],
                             p["sigma"], p["c"], p["sol"]["x"])
    xd = O.dense_solve("mhm", p["rowptr"], p["col"], p["vals"], p["n"], p["b"], p["sigma"])
    exact = sum(p["c"][k] * np.real(np.vdot(p["b"], xd[k])) for k in range(p["sigma"].size))
    assert abs(lt - exact) <= 1e-13 * abs(exact)
    # a perturbed solution x* + e: L~ - L* = -sum_k c_k e_k^H (A + sigma_k) e_k exactly,
    # while the plain loss is off by the first-order term sum_k c_k Re(b^H e_k)
    e = 1e-5 * W.gaussian_rhs(p["n"], 99, p["sigma"].size)
    xe = xd + e
    l2 = O.second_order_loss("mhm", p["rowptr"], p["col"], p["vals"], p["n"], p["b"],
                             p["sigma"], p["c"], xe)
    quad = sum(p["c"][k] * np.real(np.vdot(e[k], p["apply"](e[k], float(p["sigma"][k]))))
               for k in range(p["sigma"].size))
    first = sum(p["c"][k] * np.real(np.vdot(p["b"], e[k])) for k in range(p["sigma"].size))
    assert abs((l2 - exact) + quad) <= 1e-3 * abs(quad)
    assert abs(first) > 10.0 * abs(quad)


def test_fd_matches_dense_autograd(c3_4):
    p = c3_4
    nz = p["fd_nz"][:4]
    fd = O.fd_gradient("mhm", p["rowptr"], p["col"], p["vals"], p["n"], p["b"], p["sigma"],
                       p["c"], nz, h=1e-6)
    g = p["c"][:, None] * p["b"][None, :]
    gv_d, _ = O.dense_reference_gradient("mhm", p["rowptr"], p["col"], p["vals"], p["n"],
                                         p["b"], p["sigma"], g)
    assert _rel(fd, gv_d[nz]) < 1e-6


def test_fd_directional_matches_dense_autograd(c3_4):
    """One central difference along a random direction of every stored entry equals
    Re(sum conj(grad) delta) of the dense autograd gradient; a wrong sign or a dropped
    conjugate in either would show up here."""
    p = c3_4
    delta = W.gaussian_rhs(p["vals"].size, 6004)
    d = O.fd_directional("mhm", p["rowptr"], p["col"], p["vals"], p["n"], p["b"], p["sigma"],
                         p["c"], delta, h=1e-6)
    g = p["c"][:, None] * p["b"][None, :]
    gv_d, _ = O.dense_reference_gradient("mhm", p["rowptr"], p["col"], p["vals"], p["n"],
                                         p["b"], p["sigma"], g)
    ref = float(np.real(np.vdot(gv_d, delta)))
    assert abs(d - ref) <= 1e-6 * abs(ref)
    # the imaginary direction probes the other half of the convention
    d_i = O.fd_directional("mhm", p["rowptr"], p["col"], p["vals"], p["n"], p["b"], p["sigma"],
                           p["c"], 1j * delta, h=1e-6)
    ref_i = float(np.real(np.vdot(gv_d, 1j * delta)))
    assert abs(d_i - ref_i) <= 1e-6 * abs(ref_i)


def test_fd_directional_fixture_16x4_matches_its_recipe():
    """The stored 16^4 directional fixture names the seeds and step of its recipe."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "fd_c3_16x4_dir.json")
    rec = json.load(open(path))
    cfg = W.CONFIGS["c3_16"]
    assert rec["seeds"] == dict(links=cfg["seed_links"], b=cfg["seed_b"], c=cfg["seed_c"],
                                direction=cfg["seed_dir"])
    assert rec["h"] == cfg["fd_h"] and rec["dims"] == list(cfg["dims"])
    assert np.isfinite(rec["directional_derivative"])


@pytest.mark.parametrize("name,fixture", [("c3", "fd_c3_8x4.json"), ("c3_16", "fd_c3_16x4.json")])
def test_closed_form_matches_fd_fixture(name, fixture):
    """The oracle's closed-form gradient at 8^4 and 16^4 against the stored central
    differences (tests/golden, written by make_fd_golden.py from the oracle's FD)."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", fixture)
    rec = json.load(open(path))
    p = W.make_config(name)
    assert rec["nz"] == [int(e) for e in p["fd_nz"]]
    ap = O.shifted_apply("mhm", p["rowptr"], p["col"], p["vals"], p["n"])
    sol = O.cg_m(ap, p["b"], p["sigma"], tol=1e-14, max_iter=100000)
    gv, _ = O.closed_form_gradient("mhm", p["rowptr"], p["col"], p["vals"], p["n"], sol["x"], p["c"])
    fd = np.array(rec["grad_re"]) + 1j * np.array(rec["grad_im"])
    got = gv[np.array(rec["nz"])]
    comp_got = np.concatenate([got.real, got.imag])
    comp_fd = np.concatenate([fd.real, fd.imag])
    # Error of a central difference in floating point: each of the two loss values carries
    # a rounding error of about u |L| (u = 2^-53), so their quotient carries u |L| / h:
    # 9e-4 at 16^4, where |L| ~ 4e6, against gradients of order 1e2; the truncation error,
    # of order h^2 times the third derivative, is far below it.  Each component may differ
    # by 4 u |L| / h plus 1e-7 of the largest component.
    L = O.second_order_loss("mhm", p["rowptr"], p["col"], p["vals"], p["n"], p["b"], p["sigma"],
                            p["c"], sol["x"])
    assert abs(L - rec["loss"]) <= 1e-12 * abs(L)
    bound = 4 * 2.0 ** -53 * abs(L) / rec["h"] + 1e-7 * np.abs(comp_fd).max()
    assert np.all(np.abs(comp_got - comp_fd) <= bound)
    assert np.linalg.norm(comp_got - comp_fd) / np.linalg.norm(comp_fd) <= 2e-6
