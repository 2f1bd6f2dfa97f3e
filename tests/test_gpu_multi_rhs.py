"""GPU: a different right-hand side per shift (msc_solve_multi_rhs), through the C ABI.

Section 5, eq. linprobgen: initial guesses that leave every shifted system the same
residual, then one multishift solve.  Checked against dense solves of each
(A + sigma_k) x_k = b_k at 4^4 (staggered M^H M, FP64 and mixed), a Hermitian Laplacian,
the oracle's guesses (closed-form cases: equal right-hand sides, right-hand sides linear
in the shift), and the fallback when the guesses grow beyond FP64's reach (many shifts
over several decades) or the shifts repeat.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.linalg.norm(a - b, axis=-1) / np.linalg.norm(b, axis=-1)


@pytest.fixture(scope="module")
def stag():
    p = W.staggered_problem((4, 4, 4, 4), 0.3, 1000, 2000, (0.05, 1.0, 4))
    p["apply"] = O.shifted_apply("mhm", p["rowptr"], p["col"], p["vals"], p["n"])
    p["B"] = np.stack([W.gaussian_rhs(p["n"], 3000 + k) for k in range(p["sigma"].size)])
    p["dense"] = np.stack([O.dense_solve("mhm", p["rowptr"], p["col"], p["vals"], p["n"],
                                         p["B"][k], [s])[0] for k, s in enumerate(p["sigma"])])
    return p


def _op(p, cuda, kind="mhm"):
    from paper_1102_2143_amd import Operator
    return Operator(p["rowptr"], p["col"], p["vals"], p["n"], kind=kind, device=cuda)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_distinct_rhs_match_dense_solves(stag, cuda, prec):
    print(f"[gpu] multi-rhs 4^4 {prec}", flush=True)
    op = _op(stag, cuda)
    sig = stag["sigma"][[2, 0, 3, 1]]   # caller order is kept
    B = stag["B"][[2, 0, 3, 1]]
    dense = stag["dense"][[2, 0, 3, 1]]
    op.set_shifts(sig)
    x, info = op.solve_multi_rhs(B, tol=1e-10, prec=prec)
    assert info["status"] == "ok"
    assert info["iters"] > 0  # the common-residual multishift solve ran
    assert np.all(info["true_rel_res"] <= 1e-10)
    assert np.all(_rel(x.cpu().numpy(), dense) <= 1e-8)
    # the oracle's finished solve needs the same number of multishift iterations, +-2
    if prec == "fp64":
        ref = O.multi_rhs_solve(stag["apply"], B, sig, tol=1e-10)
        assert abs(info["iters"] - ref["iters"]) <= 2
    op.close()


def test_equal_rhs_reduce_to_the_multishift_solve(stag, cuda):
    op = _op(stag, cuda)
    op.set_shifts(stag["sigma"])
    B = np.stack([stag["b"]] * stag["sigma"].size)
    x, info = op.solve_multi_rhs(B, tol=1e-10)
    x1, info1 = op.solve(stag["b"], tol=1e-10)
    assert info["status"] == "ok"
    assert info["iters"] == info1["iters"]
    assert np.all(_rel(x.cpu().numpy(), x1.cpu().numpy()) <= 1e-12)
    op.close()


def test_rhs_linear_in_the_shift(stag, cuda):
    # b_k = c + sigma_k d: the guesses are x0_k = d and r0 = c - A d (closed form)
    c, d = stag["B"][0], stag["B"][1]
    sig = stag["sigma"]
    B = np.stack([c + s * d for s in sig])
    op = _op(stag, cuda)
    op.set_shifts(sig)
    x, info = op.solve_multi_rhs(B, tol=1e-10)
    dense = np.stack([O.dense_solve("mhm", stag["rowptr"], stag["col"], stag["vals"], stag["n"],
                                    B[k], [s])[0] for k, s in enumerate(sig)])
    assert info["status"] == "ok"
    assert np.all(_rel(x.cpu().numpy(), dense) <= 1e-8)
    op.close()


def test_laplacian(cuda):
    rowptr, col, vals = W.laplacian7_csr((9, 8, 7), 41)
    p = dict(rowptr=rowptr, col=col, vals=vals, n=504)
    sig = np.array([0.3, 0.05, 0.8])
    B = np.stack([W.gaussian_rhs(504, 50 + k) for k in range(3)])
    op = _op(p, cuda, kind="herm")
    op.set_shifts(sig)
    x, info = op.solve_multi_rhs(B, tol=1e-10)
    dense = np.stack([O.dense_solve("herm", rowptr, col, vals, 504, B[k], [s])[0]
                      for k, s in enumerate(sig)])
    assert info["status"] == "ok"
    assert np.all(_rel(x.cpu().numpy(), dense) <= 1e-8)
    op.close()


def test_fallback_when_the_guesses_grow_or_shifts_repeat(stag, cuda):
    # ten shifts over four decades: |r0| / |b| ~ 1e23, beyond FP64; repeated shifts have
    # no common residual.  Every shift is then solved from zero by the batched CG.
    op = _op(stag, cuda)
    for sig in (W.logspace_shifts(1e-3, 1.0, 10), np.array([0.2, 0.5, 0.2])):
        B = np.stack([W.gaussian_rhs(stag["n"], 70 + k) for k in range(sig.size)])
        op.set_shifts(sig)
        x, info = op.solve_multi_rhs(B, tol=1e-10)
        dense = np.stack([O.dense_solve("mhm", stag["rowptr"], stag["col"], stag["vals"],
                                        stag["n"], B[k], [s])[0] for k, s in enumerate(sig)])
        assert info["status"] == "ok"
        assert info["iters"] == 0 and info["refine_iters"] > 0
        assert np.all(_rel(x.cpu().numpy(), dense) <= 1e-8)
    op.close()
