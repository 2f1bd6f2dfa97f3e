"""Pins of the BiCGStab-M oracle (CPU only).

The multishift BiCGStab is derived in oracle/bicgstab.py from the BiCG polynomials (the
paper names BiCGStab-M as its second solver, Sections 1 and 3, but prints only CG-M).
Its pins, none of which re-uses the oracle's own recurrences:

* the plain definition x_k = (A + sigma_k)^{-1} b by a dense LAPACK solve, for the
  non-Hermitian staggered M itself (the multi-mass Dirac system (M + sigma_k) x = b) and
  for a random non-Hermitian sparse matrix with empty rows;
* one shift: the iterates equal textbook BiCGStab's (van der Vorst's method written
  plainly) step by step;
* collinearity: b - (A + sigma_k) x_k^(n) = (z_n / tau_n) r_n for every n (the shifted
  residual is the driving one scaled);
* duplicates and caller order; b = 0.
Planted mistakes in the shifted constants each fail at least one pin.
"""
import importlib
import inspect
import types

import numpy as np
import pytest

import oracle as O
import workloads as W


def _rel(a, b):
    return np.linalg.norm(a - b, axis=-1) / np.linalg.norm(b, axis=-1)


@pytest.fixture(scope="module")
def stag():
    # M = m + D on 4^4 (non-Hermitian: D is anti-Hermitian); shifts add to the mass
    p = W.staggered_problem((4, 4, 4, 4), 0.1, 1000, 2000, (1e-2, 1.0, 6))
    p["apply"] = O.shifted_apply("general", p["rowptr"], p["col"], p["vals"], p["n"])
    p["dense"] = O.dense_solve("general", p["rowptr"], p["col"], p["vals"], p["n"], p["b"],
                               p["sigma"])
    return p


def test_dense_solve_staggered_m(stag):
    res = O.bicgstab_m(stag["apply"], stag["b"], stag["sigma"], tol=1e-11)
    assert res["status"] == "ok"
    assert np.all(res["true_rel_res"] <= 1e-10)
    assert np.all(_rel(res["x"], stag["dense"]) <= 1e-9)


def test_dense_solve_random_nonhermitian_with_empty_rows():
    n = 300
    rowptr, col, vals = W.random_sparse_csr(n, 21, 7, diag=4.0 + 1.0j, empty_rows=(3, 99))
    # empty rows make A singular; the shifts (>= 0.5) make every A + sigma invertible
    b = W.gaussian_rhs(n, 8)
    sigma = np.array([0.5, 0.8, 1.5, 3.0])
    ap = O.shifted_apply("general", rowptr, col, vals, n)
    res = O.bicgstab_m(ap, b, sigma, tol=1e-12)
    dense = O.dense_solve("general", rowptr, col, vals, n, b, sigma)
    assert res["status"] == "ok"
    assert np.all(_rel(res["x"], dense) <= 1e-9)


def test_one_shift_is_textbook_bicgstab(stag):
    ap, b = stag["apply"], stag["b"]
    for shift in (0.0, 0.3):
        ref = O.bicgstab(ap, b, shift=shift, tol=0.0, max_iter=25, record=True)["history"]
        got = []

        def observe(n, r, shifts):
            got.append(shifts[0].x.copy())

        O.bicgstab_m(ap, b, [shift], tol=0.0, max_iter=25, observe=observe, verify=False)
        assert len(got) == 25
        for n in range(1, 26):
            assert np.linalg.norm(got[n - 1] - ref[n]) <= 1e-12 * np.linalg.norm(ref[n])


def test_shifted_residuals_are_collinear(stag):
    ap, b, sigma = stag["apply"], stag["b"], stag["sigma"]
    bn = np.linalg.norm(b)
    order = np.argsort(sigma, kind="stable")
    worst = [0.0]

    def observe(n, r, shifts):
        for j, sh in enumerate(shifts):
            res = b - ap(sh.x, float(sigma[order[j]]))
            worst[0] = max(worst[0], np.linalg.norm(res - (sh.z / sh.tau) * r) / bn)

    O.bicgstab_m(ap, b, sigma, tol=0.0, max_iter=60, observe=observe, verify=False)
    assert worst[0] <= 1e-10


def test_duplicates_order_and_zero_rhs(stag):
    ap, b = stag["apply"], stag["b"]
    sig = np.array([0.5, 0.05, 0.5, 0.2])
    res = O.bicgstab_m(ap, b, sig, tol=1e-10)
    assert np.array_equal(res["x"][0], res["x"][2])
    ref = O.bicgstab_m(ap, b, np.sort(sig), tol=1e-10)
    assert np.allclose(res["x"][1], ref["x"][0], rtol=0, atol=1e-13 * np.abs(ref["x"][0]).max())
    zero = O.bicgstab_m(ap, np.zeros_like(b), sig)
    assert zero["status"] == "ok" and zero["iters"] == 0 and not zero["x"].any()


MUTANTS = {
    "unscaled stabilising step": ("om_s = om / g", "om_s = om"),
    "power of the ratio in be(s)": ("be * (sh.z_new / sh.z) ** 2", "be * (sh.z_new / sh.z)"),
    "new z in the back term": ("back = (sh.z / sh.tau) * r", "back = (sh.z_new / sh.tau) * r"),
    "tau not advanced": ("tau_new = sh.tau * g", "tau_new = sh.tau"),
    "denominator sign": ("* (1.0 + sh.s * al)", "* (1.0 - sh.s * al)"),
    "old tau in the new direction": ("(sh.z_new / tau_new) * r_new", "(sh.z_new / sh.tau) * r_new"),
}


def _mutant(old, new):
    # the module itself (the package re-exports its function under the same name)
    src = inspect.getsource(importlib.import_module("oracle.bicgstab"))
    assert src.count(old) == 1, old
    mod = types.ModuleType("bicgstab_mutant")
    exec(compile(src.replace(old, new), "bicgstab_mutant", "exec"), mod.__dict__)
    return mod.bicgstab_m


def _failed_pins(fn, p):
    ap, b, sigma = p["apply"], p["b"], p["sigma"]
    failed = []
    with np.errstate(all="ignore"):
        try:
            res = fn(ap, b, sigma, tol=1e-11, max_iter=3000)
            if not (res["status"] == "ok" and np.all(_rel(res["x"], p["dense"]) <= 1e-9)):
                failed.append("dense")
        except Exception:
            failed.append("dense")
        try:
            bn = np.linalg.norm(b)
            order = np.argsort(sigma, kind="stable")
            worst = [0.0]

            def observe(n, r, shifts):
                for j, sh in enumerate(shifts):
                    res_k = b - ap(sh.x, float(sigma[order[j]]))
                    worst[0] = max(worst[0], np.linalg.norm(res_k - (sh.z / sh.tau) * r) / bn)

            fn(ap, b, sigma, tol=0.0, max_iter=40, observe=observe, verify=False)
            if not worst[0] <= 1e-10:
                failed.append("collinearity")
        except Exception:
            failed.append("collinearity")
    return failed


def test_real_oracle_passes_the_mutant_pins(stag):
    assert _failed_pins(O.bicgstab_m, stag) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_fails_a_pin(stag, name):
    old, new = MUTANTS[name]
    assert _failed_pins(_mutant(old, new), stag), name
