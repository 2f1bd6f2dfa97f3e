"""torch.autograd wiring of the multishift solve and its hand-written adjoint.

``multishift_solve(vals, b, op, **params)`` returns x of shape (ns, n) with
x_k = (A(vals) + sigma_k I)^{-1} b.  Its backward calls ``msc_solve_adjoint``, which
solves y_k = (A + sigma_k)^{-1} g_k on the GPU and forms
grad_b = sum_k y_k and, for A = M^H M, the gradient with respect to M's stored values
-sum_k [(M y_k)_i conj(x_k)_j + (M x_k)_i conj(y_k)_j] (torch's complex convention).

The operator is shared state: its values and shifts may change between a forward and
its backward (another forward on the same operator, ``update_values``, ``set_shifts``).
Each forward therefore keeps its own values (the autograd input itself, not a copy) and
shifts, and a backward that finds the operator changed puts them back for its adjoint
solve, then restores the operator's later state.
"""
from __future__ import annotations

import torch

from .api import Operator


def _load_state(op: Operator, vals, sigma):
    op.update_values(vals)
    op.set_shifts(sigma)


class MultiShiftSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vals, b, op: Operator, params: dict):
        v = vals.detach()
        op.update_values(v)
        x, info = op.solve(b.detach(), **params)
        if info["status"] != "ok":
            raise RuntimeError(f"multishift solve did not converge: {info['status']}")
        op._autograd_vals = v          # the values the operator now holds
        ctx.op = op
        ctx.params = params
        ctx.sigma = op.sigma.copy()
        ctx.version = op.version
        ctx.save_for_backward(x, v)
        ctx.vals_needs = vals.requires_grad
        ctx.b_needs = b.requires_grad
        return x

    @staticmethod
    def backward(ctx, gx):
        x, vals = ctx.saved_tensors
        op = ctx.op
        changed = op.version != ctx.version
        later = None
        if changed:
            # the operator moved on since this forward: remember what it holds now (the
            # values of a later forward are known; values uploaded otherwise are not
            # kept by the binding), then differentiate at this forward's state
            later_vals = getattr(op, "_autograd_vals", None)
            later = (later_vals, None if op.sigma is None else op.sigma.copy())
            _load_state(op, vals, ctx.sigma)
        try:
            gb, gv, info = op.solve_adjoint(gx.contiguous(), x, grad_vals=ctx.vals_needs,
                                            grad_b=ctx.b_needs, **ctx.params)
        finally:
            if changed:
                later_vals, later_sigma = later
                if later_vals is not None and later_sigma is not None:
                    _load_state(op, later_vals, later_sigma)
                    op._autograd_vals = later_vals
                else:
                    # nothing to go back to: the operator keeps this forward's state
                    op._autograd_vals = vals
        if info["status"] not in ("ok",):
            raise RuntimeError(f"adjoint solve did not converge: {info['status']}")
        return gv, gb, None, None


def multishift_solve(vals, b, op: Operator, **params):
    """Differentiable x = [(A(vals) + sigma_k)^{-1} b]_k; see the module docstring."""
    return MultiShiftSolve.apply(vals, b, op, params)
