"""Python binding of the C ABI: argument marshalling only.

Device memory and streams come from torch; every numerical step runs in ``libmsc.so``.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L

_PREC = {"fp64": L.MSC_PREC_FP64, "mixed": L.MSC_PREC_MIXED}
_KIND = {"mhm": L.MSC_A_MHM, "herm": L.MSC_A_HERM, "general": L.MSC_A_GENERAL}
_FORMAT = {"auto": L.MSC_FORMAT_AUTO, "csr": L.MSC_FORMAT_CSR, "sell": L.MSC_FORMAT_SELL,
           "sell32": L.MSC_FORMAT_SELL32, "stencil": L.MSC_FORMAT_STENCIL}


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev_tensor(a, dtype, device):
    if isinstance(a, torch.Tensor):
        t = a.to(device=device, dtype=dtype)
    else:
        t = torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dtype)
    return t.contiguous()


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


def _numel(a) -> int:
    """Element count of a tensor or array-like without moving it."""
    if isinstance(a, torch.Tensor):
        return int(a.numel())
    return int(np.asarray(a).size)


def _need(cond, msg):
    # the C ABI sees raw pointers only: every length is checked here before a call
    if not cond:
        raise ValueError(msg)


def _check_out(out, shape, device, what):
    """`out` must be a contiguous complex128 tensor of `shape` on `device`."""
    _need(isinstance(out, torch.Tensor), f"{what}: out must be a torch tensor")
    _need(tuple(out.shape) == tuple(shape),
          f"{what}: out has shape {tuple(out.shape)}, expected {tuple(shape)}")
    _need(out.dtype == torch.complex128, f"{what}: out must be complex128, got {out.dtype}")
    _need(out.device == device, f"{what}: out is on {out.device}, the operator on {device}")
    _need(out.is_contiguous(), f"{what}: out must be contiguous")


_SWEEP = {"auto": 0, "contiguous": 1}


def make_params(tol=1e-10, prec="fp64", max_iter=10000, reliable_every=50, freeze=True,
                refine=True, poll_every=16, switch_tol=None, refine_max_iter=10000, lanes=0,
                verify=True, timing=0, max_grid=0, format="auto", mixed_margin=None,
                update_steps=None, sweep="auto") -> L.Params:
    lib = L.load()
    p = L.Params()
    lib.msc_params_default(ctypes.byref(p))
    p.tol = float(tol)
    p.prec = _PREC[prec] if isinstance(prec, str) else int(prec)
    p.max_iter = int(max_iter)
    p.reliable_every = int(reliable_every)
    p.freeze = int(bool(freeze))
    p.refine = int(bool(refine))
    p.poll_every = int(poll_every)
    if switch_tol is not None:
        p.switch_tol = float(switch_tol)
    p.refine_max_iter = int(refine_max_iter)
    p.lanes = int(lanes)
    p.verify = int(bool(verify))
    p.timing = int(timing)
    p.max_grid = int(max_grid)
    p.format = _FORMAT[format] if isinstance(format, str) else int(format)
    if mixed_margin is not None:
        p.mixed_margin = float(mixed_margin)
    if update_steps is not None:
        p.update_steps = int(update_steps)
    p.sweep = _SWEEP[sweep] if isinstance(sweep, str) else int(sweep)
    return p


class Operator:
    """A CSR operator resident on the GPU: A = M^H M (kind "mhm"), a Hermitian positive
    definite A itself ("herm"), or any A ("general", solved by solve_bicgstab)."""

    def __init__(self, rowptr, col, vals, n, kind="mhm", device="cuda:0", stream=None):
        self.n = int(n)
        self.kind = kind
        self.sigma = None
        self.version = 0      # bumped whenever the values or the shifts change
        self._autograd_vals = None  # values of the last autograd forward, while current
        self.handle = None
        _need(kind in _KIND, f"unknown operator kind {kind!r}")
        _need(self.n >= 1, "n must be >= 1")
        _need(_numel(rowptr) == self.n + 1,
              f"rowptr has {_numel(rowptr)} entries, expected n + 1 = {self.n + 1}")
        _need(_numel(vals) == _numel(col),
              f"vals has {_numel(vals)} entries but col has {_numel(col)}")
        self.lib = L.load()
        self.device = torch.device(device)
        rp = _dev_tensor(rowptr, torch.int64, self.device)
        cl = _dev_tensor(col, torch.int32, self.device)
        vl = _dev_tensor(vals, torch.complex128, self.device)
        self.nnz = int(cl.numel())
        h = ctypes.c_void_p()
        st = self.lib.msc_op_create_csr(ctypes.byref(h), _KIND[kind], self.n, self.nnz, _ptr(rp),
                                        _ptr(cl), _ptr(vl), _stream(stream))
        if st != L.MSC_OK:
            raise L.MscError(st, "msc_op_create_csr")
        self.handle = h

    @classmethod
    def staggered(cls, links, dims, mass, device="cuda:0", stream=None):
        """The staggered operator M = m + D from gauge links U (4, V, 3, 3) complex128:
        A = M^H M with a matrix-free multishift iteration (msc_op_create_staggered)."""
        dims = tuple(int(L) for L in dims)
        _need(len(dims) == 4, "staggered: dims must have four extents")
        _need(all(L >= 3 for L in dims), "staggered: every extent must be >= 3")
        vol = int(np.prod(dims))
        _need(_numel(links) == 4 * vol * 9,
              f"staggered: links has {_numel(links)} entries, expected 4 * V * 9 = {36 * vol}")
        self = cls.__new__(cls)
        self.n = 3 * vol
        self.kind = "mhm"
        self.sigma = None
        self.version = 0
        self._autograd_vals = None
        self.handle = None
        self.lib = L.load()
        self.device = torch.device(device)
        lk = _dev_tensor(links, torch.complex128, self.device)
        d = (ctypes.c_int32 * 4)(*dims)
        h = ctypes.c_void_p()
        st = self.lib.msc_op_create_staggered(ctypes.byref(h), d, float(mass), _ptr(lk),
                                              _stream(stream))
        if st != L.MSC_OK:
            raise L.MscError(st, "msc_op_create_staggered")
        self.handle = h
        self.nnz = 25 * self.n
        self.dims = dims
        return self

    def update_links(self, links, stream=None):
        """New gauge links for an operator made by Operator.staggered."""
        _need(_numel(links) == 12 * self.n,
              f"update_links: links has {_numel(links)} entries, expected {12 * self.n}")
        lk = _dev_tensor(links, torch.complex128, self.device)
        st = self.lib.msc_op_update_links(self.handle, _ptr(lk), _stream(stream))
        if st != L.MSC_OK:
            raise L.MscError(st, "msc_op_update_links")
        self.version += 1
        self._autograd_vals = None

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.lib.msc_op_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_shifts(self, sigma):
        s = np.ascontiguousarray(np.asarray(sigma, dtype=np.float64).reshape(-1))
        st = self.lib.msc_op_set_shifts(self.handle,
                                        s.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        int(s.size))
        if st != L.MSC_OK:
            raise L.MscError(st, "msc_op_set_shifts")
        self.sigma = s.copy()
        self.version += 1

    def storage(self):
        """{"sell": sliced ELLPACK copy built, "narrow": (matrix, M^H) copies with 16-bit
        column offsets, "two_rows": a staggered operator whose links are in SU(3), read by
        the iteration as their first two rows}."""
        sell, narrow = ctypes.c_int32(), ctypes.c_int32()
        st = self.lib.msc_op_storage(self.handle, ctypes.byref(sell), ctypes.byref(narrow))
        if st != L.MSC_OK:
            raise L.MscError(st, "msc_op_storage")
        return {"sell": bool(sell.value),
                "narrow": (bool(narrow.value & 1), bool(narrow.value & 2)),
                "two_rows": bool(narrow.value & 4)}

    def update_values(self, vals, stream=None):
        _need(_numel(vals) == self.nnz,
              f"update_values: {_numel(vals)} values, the operator has {self.nnz} entries")
        vl = _dev_tensor(vals, torch.complex128, self.device)
        st = self.lib.msc_op_update_values(self.handle, _ptr(vl), _stream(stream))
        if st != L.MSC_OK:
            raise L.MscError(st, "msc_op_update_values")
        self.version += 1
        self._autograd_vals = None

    def apply(self, v, shift=0.0, prec="fp64", stream=None):
        _need(_numel(v) == self.n, f"apply: v has {_numel(v)} entries, expected n = {self.n}")
        _need(prec in _PREC, f"apply: unknown precision {prec!r}")
        vin = _dev_tensor(v, torch.complex128, self.device).reshape(-1)
        out = torch.empty_like(vin)
        st = self.lib.msc_op_apply(self.handle, _PREC[prec], _ptr(vin), _ptr(out), float(shift),
                                   _stream(stream))
        if st != L.MSC_OK:
            raise L.MscError(st, "msc_op_apply")
        return out

    def apply_noalloc(self, v, out, shift=0.0, prec="fp64", stream=None):
        """out = (A + shift) v through msc_op_apply_noalloc: the library allocates nothing
        and only queues the work on the stream (the caller provides `out`)."""
        _need(_numel(v) == self.n, f"apply_noalloc: v has {_numel(v)} entries, expected n = {self.n}")
        _need(prec in _PREC, f"apply_noalloc: unknown precision {prec!r}")
        _check_out(out, (self.n,), self.device, "apply_noalloc")
        vin = _dev_tensor(v, torch.complex128, self.device).reshape(-1)
        st = self.lib.msc_op_apply_noalloc(self.handle, _PREC[prec], _ptr(vin), _ptr(out),
                                           float(shift), _stream(stream))
        if st != L.MSC_OK:
            raise L.MscError(st, "msc_op_apply_noalloc")
        return out

    def solve(self, b, out=None, stream=None, check=True, **kw):
        """x (ns, n) complex128 for (A + sigma_k) x_k = b; returns (x, info dict)."""
        if self.sigma is None:
            raise ValueError("set_shifts first")
        ns = self.sigma.size
        _need(_numel(b) == self.n, f"solve: b has {_numel(b)} entries, expected n = {self.n}")
        if out is not None:
            _check_out(out, (ns, self.n), self.device, "solve")
        bt = _dev_tensor(b, torch.complex128, self.device)
        x = torch.empty((ns, self.n), dtype=torch.complex128, device=self.device) if out is None else out
        prm = make_params(**kw)
        info, rel, fi = _new_info(ns)
        st = self.lib.msc_solve(self.handle, _ptr(bt), _ptr(x), ctypes.byref(prm),
                                ctypes.byref(info), _stream(stream))
        res = _info_dict(st, info, rel, fi)
        if check and st not in (L.MSC_OK, L.MSC_ENOTCONV):
            raise L.MscError(st, "msc_solve")
        return x, res

    def solve_bicgstab(self, b, out=None, stream=None, check=True, **kw):
        """x (ns, n) complex128 for (A + sigma_k) x_k = b by multishift BiCGStab (general A);
        returns (x, info dict)."""
        if self.sigma is None:
            raise ValueError("set_shifts first")
        ns = self.sigma.size
        _need(_numel(b) == self.n, f"solve_bicgstab: b has {_numel(b)} entries, expected n = {self.n}")
        if out is not None:
            _check_out(out, (ns, self.n), self.device, "solve_bicgstab")
        bt = _dev_tensor(b, torch.complex128, self.device)
        x = torch.empty((ns, self.n), dtype=torch.complex128, device=self.device) if out is None else out
        prm = make_params(**kw)
        info, rel, fi = _new_info(ns)
        st = self.lib.msc_solve_bicgstab(self.handle, _ptr(bt), _ptr(x), ctypes.byref(prm),
                                         ctypes.byref(info), _stream(stream))
        res = _info_dict(st, info, rel, fi)
        if check and st not in (L.MSC_OK, L.MSC_ENOTCONV):
            raise L.MscError(st, "msc_solve_bicgstab")
        return x, res

    def solve_real(self, b, out=None, stream=None, check=True, **kw):
        """x (ns, n) float64 for a real symmetric A (kind "herm", real values): the real
        multishift path; b real of length n.  Returns (x, info dict)."""
        if self.sigma is None:
            raise ValueError("set_shifts first")
        ns = self.sigma.size
        _need(_numel(b) == self.n, f"solve_real: b has {_numel(b)} entries, expected n = {self.n}")
        if out is not None:
            _need(isinstance(out, torch.Tensor) and tuple(out.shape) == (ns, self.n)
                  and out.dtype == torch.float64 and out.device == self.device
                  and out.is_contiguous(),
                  "solve_real: out must be a contiguous float64 tensor (ns, n) on the device")
        if isinstance(b, torch.Tensor):
            _need(not b.is_complex(), "solve_real: b must be real")
        else:
            _need(not np.iscomplexobj(b), "solve_real: b must be real")
        bt = _dev_tensor(b, torch.float64, self.device)
        x = torch.empty((ns, self.n), dtype=torch.float64, device=self.device) if out is None else out
        prm = make_params(**kw)
        info, rel, fi = _new_info(ns)
        st = self.lib.msc_solve_real(self.handle, _ptr(bt), _ptr(x), ctypes.byref(prm),
                                     ctypes.byref(info), _stream(stream))
        res = _info_dict(st, info, rel, fi)
        if check and st not in (L.MSC_OK, L.MSC_ENOTCONV):
            raise L.MscError(st, "msc_solve_real")
        return x, res

    def solve_multi_rhs(self, B, out=None, stream=None, check=True, **kw):
        """x (ns, n) complex128 for (A + sigma_k) x_k = b_k with B (ns, n), one right-hand
        side per shift in the caller's shift order; returns (x, info dict)."""
        if self.sigma is None:
            raise ValueError("set_shifts first")
        ns = self.sigma.size
        _need(_numel(B) == ns * self.n,
              f"solve_multi_rhs: B has {_numel(B)} entries, expected ns * n = {ns * self.n}")
        if out is not None:
            _check_out(out, (ns, self.n), self.device, "solve_multi_rhs")
        bt = _dev_tensor(B, torch.complex128, self.device).reshape(ns, self.n)
        x = torch.empty((ns, self.n), dtype=torch.complex128, device=self.device) if out is None else out
        prm = make_params(**kw)
        info, rel, fi = _new_info(ns)
        st = self.lib.msc_solve_multi_rhs(self.handle, _ptr(bt), _ptr(x), ctypes.byref(prm),
                                          ctypes.byref(info), _stream(stream))
        res = _info_dict(st, info, rel, fi)
        if check and st not in (L.MSC_OK, L.MSC_ENOTCONV):
            raise L.MscError(st, "msc_solve_multi_rhs")
        return x, res

    def solve_adjoint(self, g, x, stream=None, grad_vals=True, grad_b=True, check=True, **kw):
        """(grad_b (n,), grad_vals (nnz,), info) of L with dL/dx = g."""
        if self.sigma is None:
            raise ValueError("set_shifts first")
        ns = self.sigma.size
        _need(_numel(g) == ns * self.n,
              f"solve_adjoint: g has {_numel(g)} entries, expected ns * n = {ns * self.n}")
        _need(_numel(x) == ns * self.n,
              f"solve_adjoint: x has {_numel(x)} entries, expected ns * n = {ns * self.n}")
        gt = _dev_tensor(g, torch.complex128, self.device).reshape(ns, self.n)
        xt = _dev_tensor(x, torch.complex128, self.device).reshape(ns, self.n)
        gb = torch.empty(self.n, dtype=torch.complex128, device=self.device) if grad_b else None
        gv = torch.empty(self.nnz, dtype=torch.complex128, device=self.device) if grad_vals else None
        prm = make_params(**kw)
        info, rel, fi = _new_info(ns)
        st = self.lib.msc_solve_adjoint(self.handle, _ptr(gt), _ptr(xt),
                                        _ptr(gb) if gb is not None else None,
                                        _ptr(gv) if gv is not None else None,
                                        ctypes.byref(prm), ctypes.byref(info), _stream(stream))
        res = _info_dict(st, info, rel, fi)
        if check and st not in (L.MSC_OK, L.MSC_ENOTCONV):
            raise L.MscError(st, "msc_solve_adjoint")
        return gb, gv, res


def _new_info(ns):
    info = L.Info()
    rel = (ctypes.c_double * ns)()
    fi = (ctypes.c_int32 * ns)()
    info.true_rel_res = ctypes.cast(rel, ctypes.POINTER(ctypes.c_double))
    info.freeze_iter = ctypes.cast(fi, ctypes.POINTER(ctypes.c_int32))
    return info, rel, fi


def _info_dict(st, info, rel, fi):
    return dict(status=L.STATUS_NAMES.get(st, st), code=int(st), iters=int(info.iters),
                refine_iters=int(info.refine_iters), n_reliable=int(info.n_reliable),
                n_refined=int(info.n_refined), true_rel_res=np.array(rel[:]),
                freeze_iter=np.array(fi[:]), seconds=float(info.seconds),
                alg_bytes=float(info.alg_bytes), kernel_ms=np.array(info.kernel_ms[:]),
                kernel_samples=int(info.kernel_samples),
                kernel_bytes=np.array(info.kernel_bytes[:]),
                fp64_kernel_ms=np.array(info.fp64_kernel_ms[:]),
                fp64_kernel_samples=int(info.fp64_kernel_samples),
                fp64_kernel_bytes=np.array(info.fp64_kernel_bytes[:]),
                iters_fp64=int(info.iters_fp64))


def solve_batched(ops, bs, stream=None, check=True, **kw):
    """Solve every op against its right-hand sides bs[s] (nrhs_s, n_s) in one call.

    Returns (xs, infos) with xs[s] of shape (nrhs_s, ns_s, n_s)."""
    _need(len(ops) == len(bs) and len(ops) >= 1,
          "solve_batched: one right-hand-side block per operator, at least one")
    for s, (op, b) in enumerate(zip(ops, bs)):
        _need(op.sigma is not None, f"solve_batched: system {s} has no shifts")
        nb = _numel(b)
        _need(nb >= op.n and nb % op.n == 0,
              f"solve_batched: system {s}: b has {nb} entries, not a multiple of n = {op.n}")
    lib = L.load()
    nsys = len(ops)
    handles = (ctypes.c_void_p * nsys)(*[op.handle.value for op in ops])
    nrhs = (ctypes.c_int32 * nsys)()
    bptr = (ctypes.c_void_p * nsys)()
    xptr = (ctypes.c_void_p * nsys)()
    keep, xs = [], []
    total = 0
    for s, (op, b) in enumerate(zip(ops, bs)):
        bt = _dev_tensor(b, torch.complex128, op.device).reshape(-1, op.n)
        nrhs[s] = bt.shape[0]
        x = torch.empty((bt.shape[0], op.sigma.size, op.n), dtype=torch.complex128, device=op.device)
        keep.append(bt)
        xs.append(x)
        bptr[s] = bt.data_ptr()
        xptr[s] = x.data_ptr()
        total += bt.shape[0]
    infos = (L.Info * total)()
    arrays = []
    t = 0
    for s, op in enumerate(ops):
        for _ in range(nrhs[s]):
            rel = (ctypes.c_double * op.sigma.size)()
            fi = (ctypes.c_int32 * op.sigma.size)()
            infos[t].true_rel_res = ctypes.cast(rel, ctypes.POINTER(ctypes.c_double))
            infos[t].freeze_iter = ctypes.cast(fi, ctypes.POINTER(ctypes.c_int32))
            arrays.append((rel, fi))
            t += 1
    prm = make_params(**kw)
    st = lib.msc_solve_batched(nsys, handles, nrhs, bptr, xptr, ctypes.byref(prm), infos,
                               _stream(stream))
    if check and st not in (L.MSC_OK, L.MSC_ENOTCONV):
        raise L.MscError(st, "msc_solve_batched")
    out = [_info_dict(st, infos[i], arrays[i][0], arrays[i][1]) for i in range(total)]
    return xs, out, L.STATUS_NAMES.get(st, st)
