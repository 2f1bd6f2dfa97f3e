"""GPU: multishift BiCGStab (msc_solve_bicgstab) against the oracle, through the C ABI.

* the non-Hermitian staggered M itself with mass shifts, (M + sigma_k) x_k = b, on 4^4:
  every shift against the oracle BiCGStab-M and against the dense solve (per-shift
  error <= 1e-8).  BiCGStab on this M (eigenvalues m +- i lambda) is so sensitive to
  rounding that its iteration count is not a function of the arithmetic alone: the
  oracle itself, applying M as a sparse or as a dense product, takes 459 and 471
  iterations, and its iterates differ by 6e-5 after five steps.  Here only what is
  unique is compared: the solutions, and true residuals below tol;
* a diagonally dominant random non-Hermitian matrix with empty rows and a Hermitian
  Laplacian, where the oracle's count does not depend on the rounding (sparse and
  dense products give the same count): iterations and freeze iterations within 2;
* one shift against textbook BiCGStab, duplicates and caller order, 64 shifts, b = 0,
  the iteration limit;
* misuse: A = M^H M operators, mixed precision, a general operator handed to CG-M.
Paper: Sections 1 and 3 (BiCGStab-M is the second shifted solver); Section 2, eq.
linprob (the family solved).
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.linalg.norm(a - b, axis=-1) / np.linalg.norm(b, axis=-1)


def _gop(rowptr, col, vals, n, cuda, kind="general"):
    from paper_1102_2143_amd import Operator
    return Operator(rowptr, col, vals, n, kind=kind, device=cuda)


@pytest.fixture(scope="module")
def stag():
    p = W.staggered_problem((4, 4, 4, 4), 0.1, 1000, 2000, (1e-2, 1.0, 8))
    p["apply"] = O.shifted_apply("general", p["rowptr"], p["col"], p["vals"], p["n"])
    p["ref"] = O.bicgstab_m(p["apply"], p["b"], p["sigma"], tol=1e-10)
    return p


def test_staggered_m_matches_oracle(stag, cuda):
    print("[gpu] bicgstab-m staggered M 4^4, 8 mass shifts", flush=True)
    op = _gop(stag["rowptr"], stag["col"], stag["vals"], stag["n"], cuda)
    op.set_shifts(stag["sigma"])
    x, info = op.solve_bicgstab(stag["b"], tol=1e-10)
    ref = stag["ref"]
    xg = x.cpu().numpy()
    print(f"[gpu] bicgstab-m iters gpu={info['iters']} oracle={ref['iters']} "
          f"max err={_rel(xg, ref['x']).max():.2e}", flush=True)
    assert info["status"] == "ok"
    assert np.all(info["true_rel_res"] <= 1e-10)
    assert np.all(_rel(xg, ref["x"]) <= 1e-8)
    dense = O.dense_solve("general", stag["rowptr"], stag["col"], stag["vals"], stag["n"],
                          stag["b"], stag["sigma"])
    assert np.all(_rel(xg, dense) <= 1e-8)
    # the library's residuals agree with the oracle's evaluation
    rho = np.array([np.linalg.norm(stag["b"] - stag["apply"](xg[k], s))
                    for k, s in enumerate(stag["sigma"])]) / np.linalg.norm(stag["b"])
    assert np.allclose(rho, info["true_rel_res"], rtol=1e-3, atol=1e-15)
    op.close()


@pytest.mark.parametrize("lanes", [4, 8, 16, 32])
def test_random_nonhermitian_with_empty_rows(cuda, lanes):
    n = 1000
    rowptr, col, vals = W.random_sparse_csr(n, 33, 11, diag=12.0 + 3.0j, empty_rows=(0, 7, 999))
    b = W.gaussian_rhs(n, 8)
    sigma = np.array([0.5, 3.0, 0.8, 1.5])
    op = _gop(rowptr, col, vals, n, cuda)
    op.set_shifts(sigma)
    x, info = op.solve_bicgstab(b, tol=1e-10, lanes=lanes)
    ap = O.shifted_apply("general", rowptr, col, vals, n)
    ref = O.bicgstab_m(ap, b, sigma, tol=1e-10)
    dense = O.dense_solve("general", rowptr, col, vals, n, b, sigma)
    assert info["status"] == "ok"
    assert np.all(info["true_rel_res"] <= 1e-10)
    assert np.all(_rel(x.cpu().numpy(), dense) <= 1e-8)
    assert abs(info["iters"] - ref["iters"]) <= 2
    assert np.all(np.abs(info["freeze_iter"] - ref["freeze_iter"]) <= 2)
    op.close()


@pytest.fixture(scope="module")
def lap():
    rowptr, col, vals = W.laplacian7_csr((10, 9, 8), 77)
    n = 720
    return dict(rowptr=rowptr, col=col, vals=vals, n=n, b=W.gaussian_rhs(n, 9),
                sigma=W.logspace_shifts(1e-3, 1.0, 5),
                apply=O.shifted_apply("herm", rowptr, col, vals, n))


def test_hermitian_laplacian(lap, cuda):
    op = _gop(lap["rowptr"], lap["col"], lap["vals"], lap["n"], cuda, kind="herm")
    op.set_shifts(lap["sigma"])
    x, info = op.solve_bicgstab(lap["b"], tol=1e-10)
    ref = O.bicgstab_m(lap["apply"], lap["b"], lap["sigma"], tol=1e-10)
    dense = O.dense_solve("herm", lap["rowptr"], lap["col"], lap["vals"], lap["n"], lap["b"],
                          lap["sigma"])
    assert info["status"] == "ok"
    assert np.all(_rel(x.cpu().numpy(), dense) <= 1e-8)
    assert abs(info["iters"] - ref["iters"]) <= 2
    op.close()


def test_one_shift_duplicates_and_order(stag, lap, cuda):
    op = _gop(stag["rowptr"], stag["col"], stag["vals"], stag["n"], cuda)
    sig = np.array([0.5, 0.05, 0.5, 0.2])
    op.set_shifts(sig)
    x, info = op.solve_bicgstab(stag["b"], tol=1e-10)
    xg = x.cpu().numpy()
    assert info["status"] == "ok"
    assert bool((x[0] == x[2]).all())
    ref = O.bicgstab_m(stag["apply"], stag["b"], sig, tol=1e-10)
    assert np.all(_rel(xg, ref["x"]) <= 1e-8)
    op.close()
    # one shift: textbook BiCGStab (on the Laplacian, whose count is rounding-stable)
    op = _gop(lap["rowptr"], lap["col"], lap["vals"], lap["n"], cuda, kind="herm")
    op.set_shifts([0.3])
    x1, info1 = op.solve_bicgstab(lap["b"], tol=1e-10)
    ref1 = O.bicgstab(lap["apply"], lap["b"], shift=0.3, tol=1e-10)
    assert abs(info1["iters"] - ref1["iters"]) <= 2
    assert _rel(x1.cpu().numpy()[0], ref1["x"]) <= 1e-8
    op.close()


def test_sixty_four_shifts(stag, cuda):
    sig = W.logspace_shifts(1e-2, 2.0, 64)
    op = _gop(stag["rowptr"], stag["col"], stag["vals"], stag["n"], cuda)
    op.set_shifts(sig)
    x, info = op.solve_bicgstab(stag["b"], tol=1e-10)
    ref = O.bicgstab_m(stag["apply"], stag["b"], sig, tol=1e-10)
    assert info["status"] == "ok"
    assert np.all(_rel(x.cpu().numpy(), ref["x"]) <= 1e-8)
    op.close()


def test_zero_rhs_and_iteration_limit(stag, lap, cuda):
    from paper_1102_2143_amd import MscError
    op = _gop(lap["rowptr"], lap["col"], lap["vals"], lap["n"], cuda, kind="herm")
    op.set_shifts(lap["sigma"])
    x, info = op.solve_bicgstab(np.zeros(lap["n"], complex), tol=1e-10)
    assert info["status"] == "ok" and info["iters"] == 0 and not bool(x.abs().max() > 0)
    # the iterates after five steps equal the oracle's
    x, info = op.solve_bicgstab(lap["b"], tol=1e-10, max_iter=5, poll_every=1)
    assert info["status"] == "notconv" and info["iters"] == 5
    ref = O.bicgstab_m(lap["apply"], lap["b"], lap["sigma"], tol=0.0, max_iter=5)
    assert np.all(_rel(x.cpu().numpy(), ref["x"]) <= 1e-12)
    op.close()
    op = _gop(stag["rowptr"], stag["col"], stag["vals"], stag["n"], cuda)
    op.set_shifts(stag["sigma"])
    with pytest.raises(MscError):
        op.solve_bicgstab(stag["b"], prec="mixed")
    with pytest.raises(MscError):
        op.solve(stag["b"])  # CG-M needs a Hermitian positive-definite A
    op.close()
    mhm = _gop(stag["rowptr"], stag["col"], stag["vals"], stag["n"], cuda, kind="mhm")
    mhm.set_shifts(stag["sigma"])
    with pytest.raises(MscError):
        mhm.solve_bicgstab(stag["b"])
    mhm.close()
