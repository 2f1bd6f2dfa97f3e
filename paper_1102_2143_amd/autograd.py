"""torch.autograd wiring of the multishift solve and its hand-written adjoint.

``multishift_solve(vals, b, op, **params)`` returns x of shape (ns, n) with
x_k = (A(vals) + sigma_k I)^{-1} b.  Its backward calls ``msc_solve_adjoint``, which
solves y_k = (A + sigma_k)^{-1} g_k on the GPU and forms
grad_b = sum_k y_k and, for A = M^H M, the gradient with respect to M's stored values
-sum_k [(M y_k)_i conj(x_k)_j + (M x_k)_i conj(y_k)_j] (torch's complex convention).
"""
from __future__ import annotations

import torch

from .api import Operator


class MultiShiftSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vals, b, op: Operator, params: dict):
        op.update_values(vals.detach())
        x, info = op.solve(b.detach(), **params)
        if info["status"] != "ok":
            raise RuntimeError(f"multishift solve did not converge: {info['status']}")
        ctx.op = op
        ctx.params = params
        ctx.save_for_backward(x)
        ctx.vals_needs = vals.requires_grad
        ctx.b_needs = b.requires_grad
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        gb, gv, info = ctx.op.solve_adjoint(gx.contiguous(), x, grad_vals=ctx.vals_needs,
                                            grad_b=ctx.b_needs, **ctx.params)
        if info["status"] not in ("ok",):
            raise RuntimeError(f"adjoint solve did not converge: {info['status']}")
        return gv, gb, None, None


def multishift_solve(vals, b, op: Operator, **params):
    """Differentiable x = [(A(vals) + sigma_k)^{-1} b]_k; see the module docstring."""
    return MultiShiftSolve.apply(vals, b, op, params)
