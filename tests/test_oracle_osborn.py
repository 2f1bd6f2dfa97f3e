"""Pins of the common-residual initial guesses (Section 5, eq. linprobgen) (CPU only).

* the defining property: b_k - (A + sigma_k) x0_k is the same vector r0 for every k,
  checked by applying A independently;
* closed forms: equal right-hand sides give x0 = 0, r0 = b; two shifts give the one
  guess (b_1 - b_0) / (sigma_1 - sigma_0) for both; right-hand sides linear in the shift,
  b_k = c + sigma_k d, give x0_k = d for all k and r0 = c - A d;
* the finished solve against dense solves with a different b_k per shift (staggered
  M^H M and a Hermitian Laplacian).
Planted mistakes in the construction each fail a pin.
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
    p = W.staggered_problem((4, 4, 4, 4), 0.3, 1000, 2000, (0.05, 1.0, 4))
    p["apply"] = O.shifted_apply("mhm", p["rowptr"], p["col"], p["vals"], p["n"])
    p["B"] = np.stack([W.gaussian_rhs(p["n"], 3000 + k) for k in range(p["sigma"].size)])
    return p


def _common_residual_error(apply_A, B, sigma, x0, r0):
    worst = 0.0
    for k in range(sigma.size):
        res = B[k] - apply_A(x0[k], float(sigma[k]))
        scale = max(np.linalg.norm(B[k]), np.linalg.norm(apply_A(x0[k], float(sigma[k]))))
        worst = max(worst, np.linalg.norm(res - r0) / scale)
    return worst


def test_every_guess_leaves_the_same_residual(stag):
    sig = stag["sigma"][[2, 0, 3, 1]]  # any caller order
    B = stag["B"]
    x0, r0 = O.common_residual_guesses(stag["apply"], B, sig)
    assert _common_residual_error(stag["apply"], B, sig, x0, r0) <= 1e-13


def test_equal_right_hand_sides_need_no_guess(stag):
    B = np.stack([stag["b"]] * 4)
    x0, r0 = O.common_residual_guesses(stag["apply"], B, stag["sigma"])
    assert not x0.any() and np.array_equal(r0, stag["b"])


def test_two_shifts_closed_form(stag):
    B, sig = stag["B"][:2], np.array([0.7, 0.2])
    x0, r0 = O.common_residual_guesses(stag["apply"], B, sig)
    y = (B[0] - B[1]) / (sig[0] - sig[1])
    assert np.allclose(x0[0], y, rtol=0, atol=1e-14 * np.abs(y).max())
    assert np.allclose(x0[1], y, rtol=0, atol=1e-14 * np.abs(y).max())
    ref = B[1] - stag["apply"](y, 0.2)
    assert np.allclose(r0, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def test_right_hand_sides_linear_in_the_shift(stag):
    c, d = stag["B"][0], stag["B"][1]
    sig = stag["sigma"]
    B = np.stack([c + s * d for s in sig])
    x0, r0 = O.common_residual_guesses(stag["apply"], B, sig)
    for k in range(sig.size):
        assert np.linalg.norm(x0[k] - d) <= 1e-12 * np.linalg.norm(d)
    ref = c - stag["apply"](d, 0.0)
    assert np.linalg.norm(r0 - ref) <= 1e-12 * np.linalg.norm(ref)


def test_finished_solve_matches_dense_solves(stag):
    res = O.multi_rhs_solve(stag["apply"], stag["B"], stag["sigma"], tol=1e-11)
    dense = np.stack([O.dense_solve("mhm", stag["rowptr"], stag["col"], stag["vals"], stag["n"],
                                    stag["B"][k], [s])[0] for k, s in enumerate(stag["sigma"])])
    assert np.all(res["true_rel_res"] <= 1e-10)
    assert np.all(_rel(res["x"], dense) <= 1e-8)


def test_finished_solve_laplacian():
    rowptr, col, vals = W.laplacian7_csr((9, 8, 7), 41)
    n = 504
    sig = np.array([0.3, 0.05, 0.8])
    B = np.stack([W.gaussian_rhs(n, 50 + k) for k in range(3)])
    ap = O.shifted_apply("herm", rowptr, col, vals, n)
    res = O.multi_rhs_solve(ap, B, sig, tol=1e-11)
    dense = np.stack([O.dense_solve("herm", rowptr, col, vals, n, B[k], [s])[0]
                      for k, s in enumerate(sig)])
    assert np.all(_rel(res["x"], dense) <= 1e-8)


def test_repeated_shift_is_rejected(stag):
    with pytest.raises(ValueError):
        O.common_residual_guesses(stag["apply"], stag["B"][:2], [0.5, 0.5])


MUTANTS = {
    "wrong node in the divided difference": ("(s[k] - s[k - level])", "(s[k] - s[k - 1])"),
    "shift of the wrong node in the recurrence": ("apply_A(Y[j], float(s[j]))",
                                                  "apply_A(Y[j], float(s[j - 1]))"),
    "Newton weight advanced before use": ("acc = acc + w * Y[j]\n            w = w * (s[kk] - s[j])",
                                          "w = w * (s[kk] - s[j])\n            acc = acc + w * Y[j]"),
    "last coefficient dropped": ("Y[m - 2] = D[m - 1].copy()", "Y[m - 2] = 0 * D[m - 1]"),
}


def _mutant(old, new):
    src = inspect.getsource(importlib.import_module("oracle.osborn"))
    assert src.count(old) == 1, old
    mod = types.ModuleType("osborn_mutant", )
    mod.__dict__["__name__"] = "oracle.osborn_mutant"
    mod.__dict__["__package__"] = "oracle"
    exec(compile(src.replace(old, new), "osborn_mutant", "exec"), mod.__dict__)
    return mod.common_residual_guesses


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_fails_a_pin(stag, name):
    old, new = MUTANTS[name]
    fn = _mutant(old, new)
    failed = []
    with np.errstate(all="ignore"):
        x0, r0 = fn(stag["apply"], stag["B"], stag["sigma"])
        if not _common_residual_error(stag["apply"], stag["B"], stag["sigma"], x0, r0) <= 1e-13:
            failed.append("common residual")
        c, d = stag["B"][0], stag["B"][1]
        B = np.stack([c + s * d for s in stag["sigma"]])
        x0, _ = fn(stag["apply"], B, stag["sigma"])
        if not all(np.linalg.norm(x0[k] - d) <= 1e-12 * np.linalg.norm(d)
                   for k in range(stag["sigma"].size)):
            failed.append("linear closed form")
    assert failed, name
