"""GPU: the hand-written adjoint against the dense autograd reference, the closed form
and central finite differences of the oracle."""
import json
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _op(p, cuda, kind="mhm"):
    from paper_1102_2143_amd import Operator
    op = Operator(p["rowptr"], p["col"], p["vals"], p["n"], kind=kind, device=cuda)
    op.set_shifts(p["sigma"])
    return op


@pytest.fixture(scope="module")
def c3_4():
    return W.make_config("c3_4")


@pytest.mark.parametrize("prec,bar", [("fp64", 1e-8), ("mixed", 1e-8)])
def test_collinear_loss_matches_dense_autograd(c3_4, cuda, prec, bar):
    print(f"[gpu] adjoint collinear 4^4 {prec}", flush=True)
    p = c3_4
    op = _op(p, cuda)
    x, info = op.solve(p["b"], tol=1e-12, prec=prec)
    g = p["c"][:, None] * p["b"][None, :]
    gb, gv, ainfo = op.solve_adjoint(g, x, tol=1e-12, prec=prec)
    assert ainfo["status"] == "ok", ainfo
    ref_v, ref_b = O.dense_reference_gradient("mhm", p["rowptr"], p["col"], p["vals"], p["n"],
                                              p["b"], p["sigma"], g)
    assert _rel(gv.cpu().numpy(), ref_v) <= bar
    assert _rel(gb.cpu().numpy(), ref_b) <= bar
    op.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_general_loss_matches_dense_autograd(c3_4, cuda, prec):
    print(f"[gpu] adjoint general 4^4 {prec}", flush=True)
    p = c3_4
    op = _op(p, cuda)
    x, _ = op.solve(p["b"], tol=1e-12, prec=prec)
    g = W.gaussian_rhs(p["n"], 91, p["sigma"].size)
    gb, gv, ainfo = op.solve_adjoint(g, x, tol=1e-12, prec=prec)
    assert ainfo["status"] == "ok", ainfo
    ref_v, ref_b = O.dense_reference_gradient("mhm", p["rowptr"], p["col"], p["vals"], p["n"],
                                              p["b"], p["sigma"], g)
    assert _rel(gv.cpu().numpy(), ref_v) <= 1e-8
    assert _rel(gb.cpu().numpy(), ref_b) <= 1e-8
    op.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_general_loss_through_one_multishift_solve(c3_4, cuda, prec):
    # four shifts a few units apart: the adjoint solves (A + sigma_k) y_k = g_k with
    # distinct g_k through the common-residual guesses (|r0| / min|g_k| ~ 25, so the
    # common residual's stop, 4e-12, stays within FP64) and one multishift solve
    # (Section 5), then completes every shift; the gradient matches dense autograd
    print(f"[gpu] adjoint general 4^4 through the multishift {prec}", flush=True)
    p = dict(c3_4)
    p["sigma"] = np.array([1.0, 4.0, 2.0, 8.0])
    op = _op(p, cuda)
    x, _ = op.solve(p["b"], tol=1e-12, prec=prec)
    g = W.gaussian_rhs(p["n"], 92, p["sigma"].size)
    g[2] = 0.0  # a zero g_k: y_k = 0
    gb, gv, ainfo = op.solve_adjoint(g, x, tol=1e-10, prec=prec)
    assert ainfo["status"] == "ok", ainfo
    assert ainfo["iters"] > 0  # the common-residual multishift solve ran
    ref_v, ref_b = O.dense_reference_gradient("mhm", p["rowptr"], p["col"], p["vals"], p["n"],
                                              p["b"], p["sigma"], g)
    assert _rel(gv.cpu().numpy(), ref_v) <= 1e-8
    assert _rel(gb.cpu().numpy(), ref_b) <= 1e-8
    op.close()


@pytest.mark.parametrize("fmt", ["auto", "csr"])
def test_herm_general_loss(cuda, fmt):
    # three shifts: the adjoint's batched CG reads the sliced copy ("auto") or CSR
    rowptr, col, vals = W.laplacian7_csr((5, 4, 6), 61)
    n = 120
    p = dict(rowptr=rowptr, col=col, vals=vals, n=n, sigma=np.array([1e-3, 0.1, 2.0]))
    b = W.gaussian_rhs(n, 62)
    op = _op(p, cuda, kind="herm")
    x, _ = op.solve(b, tol=1e-13, format=fmt)
    g = W.gaussian_rhs(n, 63, 3)
    gb, gv, ainfo = op.solve_adjoint(g, x, tol=1e-13, format=fmt)
    ref_v, ref_b = O.dense_reference_gradient("herm", rowptr, col, vals, n, b, p["sigma"], g)
    assert _rel(gv.cpu().numpy(), ref_v) <= 1e-9
    assert _rel(gb.cpu().numpy(), ref_b) <= 1e-9
    op.close()


def test_zero_gradient_gives_zero(c3_4, cuda):
    p = c3_4
    op = _op(p, cuda)
    x, _ = op.solve(p["b"], tol=1e-10)
    gb, gv, ainfo = op.solve_adjoint(np.zeros((p["sigma"].size, p["n"]), complex), x)
    assert not bool(gv.abs().max() > 0) and not bool(gb.abs().max() > 0)
    op.close()


def test_autograd_function(c3_4, cuda):
    import torch
    from paper_1102_2143_amd.autograd import multishift_solve
    p = c3_4
    op = _op(p, cuda)
    vals = torch.tensor(p["vals"], device=cuda, requires_grad=True)
    b = torch.tensor(p["b"], device=cuda, requires_grad=True)
    c = torch.tensor(p["c"], device=cuda)
    x = multishift_solve(vals, b, op, tol=1e-12)
    loss = (c * torch.real((b.detach().conj()[None, :] * x).sum(dim=1))).sum()
    gv, gb = torch.autograd.grad(loss, (vals, b))
    g = p["c"][:, None] * p["b"][None, :]
    ref_v, ref_b = O.dense_reference_gradient("mhm", p["rowptr"], p["col"], p["vals"], p["n"],
                                              p["b"], p["sigma"], g)
    assert _rel(gv.cpu().numpy(), ref_v) <= 1e-8
    assert _rel(gb.cpu().numpy(), ref_b) <= 1e-8
    op.close()


def test_autograd_two_forwards_share_one_operator(c3_4, cuda):
    # two forwards with different values (and a shift change in between) on one operator,
    # then both backwards: each gradient belongs to its own forward's A + sigma
    import torch
    from paper_1102_2143_amd.autograd import multishift_solve
    p = c3_4
    op = _op(p, cuda)
    c = torch.tensor(p["c"], device=cuda)
    rng = np.random.default_rng(77)
    vals2_np = p["vals"] * (1.0 + 0.05 * rng.standard_normal(p["vals"].size))
    sigma2 = p["sigma"] * 1.5
    v1 = torch.tensor(p["vals"], device=cuda, requires_grad=True)
    v2 = torch.tensor(vals2_np, device=cuda, requires_grad=True)
    b = torch.tensor(p["b"], device=cuda, requires_grad=True)

    def loss_of(x):
        return (c * torch.real((b.detach().conj()[None, :] * x).sum(dim=1))).sum()

    x1 = multishift_solve(v1, b, op, tol=1e-12)
    op.set_shifts(sigma2)
    x2 = multishift_solve(v2, b, op, tol=1e-12)
    g = p["c"][:, None] * p["b"][None, :]
    # backward of the first forward after the second one changed values and shifts
    gv1, gb1 = torch.autograd.grad(loss_of(x1), (v1, b))
    ref_v1, ref_b1 = O.dense_reference_gradient("mhm", p["rowptr"], p["col"], p["vals"], p["n"],
                                                p["b"], p["sigma"], g)
    assert _rel(gv1.cpu().numpy(), ref_v1) <= 1e-8
    assert _rel(gb1.cpu().numpy(), ref_b1) <= 1e-8
    # the operator is back at the second forward's state: its backward is correct too
    assert np.array_equal(op.sigma, sigma2)
    gv2, gb2 = torch.autograd.grad(loss_of(x2), (v2, b))
    ref_v2, ref_b2 = O.dense_reference_gradient("mhm", p["rowptr"], p["col"], vals2_np, p["n"],
                                                p["b"], sigma2, g)
    assert _rel(gv2.cpu().numpy(), ref_v2) <= 1e-8
    assert _rel(gb2.cpu().numpy(), ref_b2) <= 1e-8
    op.close()


@pytest.mark.parametrize("name,fixture,prec", [
    ("c3", "fd_c3_8x4.json", "fp64"), ("c3", "fd_c3_8x4.json", "mixed"),
    ("c3_16", "fd_c3_16x4.json", "fp64"), ("c3_16", "fd_c3_16x4.json", "mixed")])
def test_c3_against_finite_differences(cuda, name, fixture, prec):
    # 32 seeded stored entries, real and imaginary part each, against the oracle's
    # central differences (tests/golden, written by make_fd_golden.py from the oracle
    # only); 8^4 and 16^4, the forward and the adjoint solve in FP64 or mixed precision
    path = os.path.join(GOLDEN, fixture)
    if not os.path.exists(path):
        pytest.fail("missing golden fixture: run tests/golden/make_fd_golden.py")
    rec = json.load(open(path))
    print(f"[gpu] adjoint {name} {prec} vs oracle finite differences", flush=True)
    p = W.make_config(name)
    op = _op(p, cuda)
    x, info = op.solve(p["b"], tol=1e-12, prec=prec)
    g = p["c"][:, None] * p["b"][None, :]
    gb, gv, ainfo = op.solve_adjoint(g, x, tol=1e-12, prec=prec)
    nz = np.array(rec["nz"])
    fd = np.array(rec["grad_re"]) + 1j * np.array(rec["grad_im"])
    got = gv.cpu().numpy()[nz]
    # 64 real components, entry by entry: the central differences carry a rounding error
    # of about u |L| / h (u = 2^-53, L the loss at the unperturbed entries, stored with
    # the fixture), 5.5e-5 at 8^4 and 9e-4 at 16^4, so small entries cannot be held to a
    # relative bar of their own
    comp_got = np.concatenate([got.real, got.imag])
    comp_fd = np.concatenate([fd.real, fd.imag])
    bound = 4 * 2.0 ** -53 * abs(rec["loss"]) / rec["h"] + 1e-7 * np.abs(comp_fd).max()
    assert np.all(np.abs(comp_got - comp_fd) <= bound)
    op.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_c3_16x4_directional_derivative(cuda, prec):
    # the 16^4 gradient workload: Re(sum conj(grad) delta) of the adjoint's gradient along
    # the seeded direction over every stored entry, against the oracle's central
    # difference of the loss along that direction (tests/golden/fd_c3_16x4_dir.json)
    path = os.path.join(GOLDEN, "fd_c3_16x4_dir.json")
    if not os.path.exists(path):
        pytest.fail("missing golden fixture: run tests/golden/make_fd_golden.py directional")
    rec = json.load(open(path))
    print(f"[gpu] adjoint 16^4 {prec} vs oracle directional finite difference", flush=True)
    p = W.make_config("c3_16")
    op = _op(p, cuda)
    x, info = op.solve(p["b"], tol=1e-12, prec=prec)
    assert info["status"] == "ok", info
    g = p["c"][:, None] * p["b"][None, :]
    gb, gv, ainfo = op.solve_adjoint(g, x, tol=1e-12, prec=prec)
    assert ainfo["status"] == "ok", ainfo
    got = float(np.real(np.vdot(gv.cpu().numpy(), p["fd_dir"])))
    fd = rec["directional_derivative"]
    print(f"[gpu] adjoint 16^4 {prec}: {got:.12e} vs fd {fd:.12e}", flush=True)
    assert abs(got - fd) <= 1e-6 * abs(fd)
    op.close()
