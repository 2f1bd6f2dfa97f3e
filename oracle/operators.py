"""Sparse operators for the oracle (test infrastructure only).

The problem is the family (A + sigma_i I) x_i = b (Section 2, eq. linprob).  Three operator
kinds are supported: ``"mhm"`` where the caller gives M and A = M^H M (the lattice case,
where the fermion matrix enters through its normal operator), ``"herm"`` where the
caller gives a Hermitian positive-definite A directly, and ``"general"`` where A is any
matrix given directly (the non-Hermitian systems of BiCGStab-M).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def csr_matrix_of(rowptr, col, vals, n) -> sp.csr_matrix:
    """scipy CSR (complex128) view of the arrays (duplicates are summed by scipy)."""
    return sp.csr_matrix((np.asarray(vals, dtype=np.complex128),
                          np.asarray(col, dtype=np.int64),
                          np.asarray(rowptr, dtype=np.int64)), shape=(int(n), int(n)))


def adjoint_csr(m: sp.csr_matrix) -> sp.csr_matrix:
    """Conjugate transpose M^H as CSR with sorted columns."""
    mh = m.conj().T.tocsr()
    mh.sort_indices()
    return mh


def shifted_apply(kind: str, rowptr, col, vals, n):
    """Return ``apply(v, shift=0.0) = (A + shift I) v`` in FP64.

    kind ``"mhm"``: A v = M^H (M v); kinds ``"herm"`` and ``"general"``: A v = A v.
    """
    m = csr_matrix_of(rowptr, col, vals, n)
    if kind == "mhm":
        mh = adjoint_csr(m)

        def apply(v, shift=0.0):
            out = mh @ (m @ v)
            if shift != 0.0:
                out = out + shift * v
            return out
    elif kind in ("herm", "general"):
        def apply(v, shift=0.0):
            out = m @ v
            if shift != 0.0:
                out = out + shift * v
            return out
    else:
        raise ValueError(f"unknown operator kind {kind!r}")
    return apply
