"""Reference gradients of a loss of the shifted solutions.  Test infrastructure only.

The loss is L = sum_k Re(g_k^H x_k) with x_k = (A + sigma_k I)^{-1} b (Section 2,
eq. linprob); the RHMC use of the family (Section 2) differentiates exactly such sums.
Gradients follow torch's convention for a real loss of a complex variable z:
grad = dL/dRe(z) + i dL/dIm(z), so that dL = Re(sum conj(grad) dz).

With y_k = (A + sigma_k)^{-1} g_k (A is Hermitian):

* grad_b = sum_k y_k;
* A = M^H M, for a stored entry e = (i, j) of M:
  grad_e = -sum_k [ (M y_k)_i conj(x_k)_j + (M x_k)_i conj(y_k)_j ];
* A given directly, for a stored entry e = (i, j) of A:
  grad_e = -sum_k (y_k)_i conj(x_k)_j.

Three independent routes are provided: dense autograd through LAPACK solves, the
closed form above evaluated on oracle solutions, and central finite differences of a
second-order accurate functional.
"""
from __future__ import annotations

import math

import numpy as np

from .operators import csr_matrix_of, adjoint_csr, shifted_apply
from .cgm import cg_m


def _rows_of(rowptr):
    rowptr = np.asarray(rowptr, dtype=np.int64)
    return np.repeat(np.arange(rowptr.size - 1, dtype=np.int64), np.diff(rowptr))


def dense_reference_gradient(kind, rowptr, col, vals, n, b, sigma, g):
    """Dense torch-CPU autograd of L = sum_k Re(g_k^H x_k); returns (grad_vals, grad_b).

    ``g`` has shape (ns, n) and is held constant; b enters only through the solves.
    """
    import torch

    rows = torch.from_numpy(_rows_of(rowptr))
    cols = torch.from_numpy(np.asarray(col, dtype=np.int64))
    v = torch.tensor(np.asarray(vals, dtype=np.complex128), requires_grad=True)
    bt = torch.tensor(np.asarray(b, dtype=np.complex128), requires_grad=True)
    gt = torch.tensor(np.asarray(g, dtype=np.complex128))
    m = torch.zeros((int(n), int(n)), dtype=torch.complex128)
    m = m.index_put((rows, cols), v, accumulate=True)
    a = m.conj().T @ m if kind == "mhm" else m
    eye = torch.eye(int(n), dtype=torch.complex128)
    loss = torch.zeros((), dtype=torch.float64)
    for k, sk in enumerate(np.ravel(sigma)):
        xk = torch.linalg.solve(a + float(sk) * eye, bt)
        loss = loss + torch.real(torch.vdot(gt[k], xk))
    loss.backward()
    return v.grad.numpy().copy(), bt.grad.numpy().copy()


def adjoint_gradient(kind, rowptr, col, vals, n, x, y):
    """The closed-form gradient given forward solutions x (ns, n) and adjoint
    solutions y (ns, n); returns (grad_vals, grad_b)."""
    rows = _rows_of(rowptr)
    col = np.asarray(col, dtype=np.int64)
    x = np.asarray(x, dtype=np.complex128)
    y = np.asarray(y, dtype=np.complex128)
    grad = np.zeros(col.size, dtype=np.complex128)
    if kind == "mhm":
        m = csr_matrix_of(rowptr, col, vals, n)
        for k in range(x.shape[0]):
            u = m @ x[k]
            w = m @ y[k]
            grad -= w[rows] * np.conj(x[k][col]) + u[rows] * np.conj(y[k][col])
    else:
        for k in range(x.shape[0]):
            grad -= y[k][rows] * np.conj(x[k][col])
    return grad, y.sum(axis=0)


def closed_form_gradient(kind, rowptr, col, vals, n, x, c):
    """Gradient for g_k = c_k b: then y_k = c_k x_k (returns (grad_vals, grad_b))."""
    c = np.asarray(c, dtype=np.float64).reshape(-1, 1)
    return adjoint_gradient(kind, rowptr, col, vals, n, x, c * np.asarray(x))


def _residual_ld(kind, rowptr, col, vals, n, b, shift, x):
    """b - (A + shift) x in extended precision (numpy longdouble)."""
    rows = _rows_of(rowptr)
    col = np.asarray(col, dtype=np.int64)
    v = np.asarray(vals).astype(np.clongdouble)
    xl = np.asarray(x).astype(np.clongdouble)

    def csr_mv(rws, cls, vv, vec):
        out = np.zeros(int(n), dtype=np.clongdouble)
        np.add.at(out, rws, vv * vec[cls])
        return out

    if kind == "mhm":
        mh = adjoint_csr(csr_matrix_of(rowptr, col, vals, n))
        t = csr_mv(rows, col, v, xl)
        ax = csr_mv(_rows_of(mh.indptr), mh.indices.astype(np.int64),
                    mh.data.astype(np.clongdouble), t)
    else:
        ax = csr_mv(rows, col, v, xl)
    return np.asarray(b).astype(np.clongdouble) - ax - np.longdouble(shift) * xl


def _fsum_re_dot(u, v) -> float:
    """Re(u^H v) with a correctly rounded sum of the products."""
    prod = np.conj(u) * v
    return math.fsum(np.real(prod).astype(np.float64).tolist()) + \
        math.fsum((np.real(prod) - np.real(prod).astype(np.float64)).astype(np.float64).tolist())


def second_order_loss(kind, rowptr, col, vals, n, b, sigma, c, x):
    """L~ = sum_k c_k Re(b^H x_k + x_k^H r_k), r_k = b - (A + sigma_k) x_k.

    For the exact solutions L~ = sum_k c_k Re(b^H x_k); for approximate ones the error
    is -sum_k c_k e_k^H (A + sigma_k) e_k, second order in the solve error e_k.
    """
    bl = np.asarray(b).astype(np.clongdouble)
    total = 0.0
    for k, sk in enumerate(np.ravel(sigma)):
        xl = np.asarray(x[k]).astype(np.clongdouble)
        rk = _residual_ld(kind, rowptr, col, vals, n, b, float(sk), x[k])
        total += float(c[k]) * (_fsum_re_dot(bl, xl) + _fsum_re_dot(xl, rk))
    return total


def fd_gradient(kind, rowptr, col, vals, n, b, sigma, c, nz, h=1e-6, tol=1e-14,
                max_iter=100000):
    """Central differences of L = sum_k c_k Re(b^H x_k) with respect to the real and
    imaginary parts of the stored entries ``nz``; returns complex grad[len(nz)]."""
    vals = np.asarray(vals, dtype=np.complex128)
    out = np.zeros(len(nz), dtype=np.complex128)

    def loss(v):
        apply = shifted_apply(kind, rowptr, col, v, n)
        sol = cg_m(apply, b, sigma, tol=tol, max_iter=max_iter)
        return second_order_loss(kind, rowptr, col, v, n, b, sigma, c, sol["x"])

    for t, e in enumerate(nz):
        parts = []
        for unit in (1.0, 1j):
            vp = vals.copy()
            vm = vals.copy()
            vp[e] += unit * h
            vm[e] -= unit * h
            parts.append((loss(vp) - loss(vm)) / (2.0 * h))
        out[t] = parts[0] + 1j * parts[1]
    return out


def fd_directional(kind, rowptr, col, vals, n, b, sigma, c, delta, h=1e-6, tol=1e-14,
                   max_iter=100000):
    """Central difference of L = sum_k c_k Re(b^H x_k) along a direction of all stored
    entries: (L(v + h delta) - L(v - h delta)) / (2h), which equals
    sum_e Re(conj(grad_e) delta_e) in the convention above, to O(h^2)."""
    vals = np.asarray(vals, dtype=np.complex128)
    delta = np.asarray(delta, dtype=np.complex128)

    def loss(v):
        apply = shifted_apply(kind, rowptr, col, v, n)
        sol = cg_m(apply, b, sigma, tol=tol, max_iter=max_iter)
        return second_order_loss(kind, rowptr, col, v, n, b, sigma, c, sol["x"])

    return (loss(vals + h * delta) - loss(vals - h * delta)) / (2.0 * h)
