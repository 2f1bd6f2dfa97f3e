"""GPU: the real-valued multishift solve (msc_solve_real) against the oracle.

The paper's benchmark matrix (Section 4, Table 1) is the real 2-D 5-point Poisson
operator; the real path runs the same recurrences on real vectors and a real copy of the
matrix.  Checked: FP64 against the oracle CG-M (per-shift error <= 1e-8, iterations and
freeze iterations within 2) and against the closed-form spectrum bound; the single-
precision path at the paper's tol 1e-5 against the exact solution within kappa_k rho_k;
agreement with the complex path on the same operator; a 300 x 300 grid; the rejections
(imaginary parts, kind M^H M) and a value update.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.linalg.norm(a - b, axis=-1) / np.linalg.norm(b, axis=-1)


def _poisson(nx, ny, ns=15):
    rowptr, col, vals = W.poisson5pt_csr(nx, ny)
    n = nx * ny
    b = np.random.default_rng(77).standard_normal(n)
    sigma = W.logspace_shifts(1e-3, 1.0, ns)
    ap = O.shifted_apply("herm", rowptr, col, vals, n)
    # Dirichlet 5-point spectrum: 4 - 2 cos(pi i/(nx+1)) - 2 cos(pi j/(ny+1))
    lmin = 4 - 2 * np.cos(np.pi / (nx + 1)) - 2 * np.cos(np.pi / (ny + 1))
    lmax = 4 + 2 * np.cos(np.pi / (nx + 1)) + 2 * np.cos(np.pi / (ny + 1))
    return dict(rowptr=rowptr, col=col, vals=vals, n=n, b=b, sigma=sigma, apply=ap,
                kappa=(lmax + sigma) / (lmin + sigma))


@pytest.fixture(scope="module")
def small():
    return _poisson(30, 24)


def _op(p, cuda, kind="herm"):
    from paper_1102_2143_amd import Operator
    return Operator(p["rowptr"], p["col"], p["vals"], p["n"], kind=kind, device=cuda)


def test_fp64_matches_oracle(small, cuda):
    print("[gpu] real fp64 poisson 30x24", flush=True)
    op = _op(small, cuda)
    op.set_shifts(small["sigma"])
    x, info = op.solve_real(small["b"], tol=1e-10, prec="fp64")
    ref = O.cg_m(small["apply"], small["b"].astype(complex), small["sigma"], tol=1e-10)
    xg = x.cpu().numpy()
    assert info["status"] == "ok"
    assert np.all(info["true_rel_res"] <= 1e-10)
    assert np.all(_rel(xg, ref["x"].real) <= 1e-8)
    assert np.abs(ref["x"].imag).max() == 0.0
    assert abs(info["iters"] - ref["iters"]) <= 2
    assert np.all(np.abs(info["freeze_iter"] - ref["freeze_iter"]) <= 2)
    op.close()


def test_single_precision_at_the_papers_tolerance(small, cuda):
    # the paper's single-precision column at its tol 1e-5: every shift within the error
    # bound kappa_k rho_k of the exact solution
    op = _op(small, cuda)
    op.set_shifts(small["sigma"])
    x, info = op.solve_real(small["b"], tol=1e-5, prec="mixed")
    dense = O.dense_solve("herm", small["rowptr"], small["col"], small["vals"], small["n"],
                          small["b"].astype(complex), small["sigma"]).real
    rho = info["true_rel_res"]
    err = _rel(x.cpu().numpy(), dense)
    assert info["status"] == "ok"
    assert np.all(rho <= 1e-5)
    assert np.all(err <= small["kappa"] * rho * 1.01 + 1e-7)
    ref = O.cg_m(small["apply"], small["b"].astype(complex), small["sigma"], tol=1e-5)
    assert abs(info["iters"] - ref["iters"]) <= 2
    op.close()


def test_real_and_complex_paths_agree(small, cuda):
    op = _op(small, cuda)
    op.set_shifts(small["sigma"])
    xr, ir = op.solve_real(small["b"], tol=1e-10)
    xc, ic = op.solve(small["b"].astype(complex), tol=1e-10)
    assert abs(ir["iters"] - ic["iters"]) <= 2
    assert np.all(_rel(xr.cpu().numpy(), xc.cpu().numpy().real) <= 1e-9)
    op.close()


def test_larger_grid(cuda):
    p = _poisson(300, 300, ns=8)
    print("[gpu] real fp64 poisson 300x300", flush=True)
    op = _op(p, cuda)
    op.set_shifts(p["sigma"])
    x, info = op.solve_real(p["b"], tol=1e-10)
    ref = O.cg_m(p["apply"], p["b"].astype(complex), p["sigma"], tol=1e-10)
    assert info["status"] == "ok"
    assert np.all(_rel(x.cpu().numpy(), ref["x"].real) <= 1e-8)
    assert abs(info["iters"] - ref["iters"]) <= 2
    op.close()


def test_rejections_and_value_update(small, cuda):
    from paper_1102_2143_amd import MscError
    op = _op(small, cuda)
    op.set_shifts(small["sigma"])
    # new values, still real: the real copies follow
    vals2 = small["vals"] * 1.5
    op.update_values(vals2)
    x, info = op.solve_real(small["b"], tol=1e-10)
    ap2 = O.shifted_apply("herm", small["rowptr"], small["col"], vals2, small["n"])
    ref = O.cg_m(ap2, small["b"].astype(complex), small["sigma"], tol=1e-10)
    assert np.all(_rel(x.cpu().numpy(), ref["x"].real) <= 1e-8)
    # an imaginary part anywhere: rejected
    vals3 = vals2.copy()
    vals3[5] += 1e-3j
    op.update_values(vals3)
    with pytest.raises(MscError):
        op.solve_real(small["b"])
    op.close()
    mhm = _op(small, cuda, kind="mhm")
    mhm.set_shifts(small["sigma"])
    with pytest.raises(MscError):
        mhm.solve_real(small["b"])
    mhm.close()
