"""Generic (non-lattice) inputs: a 3-D 7-point Laplacian, random sparse matrices,
complex Gaussian right-hand sides and log-spaced shifts."""
from __future__ import annotations

import numpy as np


def logspace_shifts(lo: float, hi: float, ns: int) -> np.ndarray:
    """``ns`` shifts log-spaced in [lo, hi], both ends included."""
    return np.logspace(np.log10(lo), np.log10(hi), int(ns))


def gaussian_rhs(n: int, seed: int, count: int | None = None) -> np.ndarray:
    """Complex Gaussian vector(s) with E|b_i|^2 = 1: (N(0,1) + i N(0,1)) / sqrt(2)."""
    rng = np.random.default_rng(seed)
    shape = (int(n),) if count is None else (int(count), int(n))
    g = rng.standard_normal(shape + (2,))
    return np.ascontiguousarray((g[..., 0] + 1j * g[..., 1]) / np.sqrt(2.0))


def laplacian7_csr(dims, seed: int, diag_lo: float = 0.01, diag_hi: float = 1.0):
    """3-D 7-point Laplacian with Dirichlet boundaries plus a random diagonal.

    Entries: ``6 + u_i`` on the diagonal with ``u_i ~ U(diag_lo, diag_hi)`` and ``-1`` for
    each in-grid neighbour; stored as complex128 with zero imaginary part.  The matrix is
    real symmetric positive definite, so it is given to the solver directly as A.
    Sites are numbered ``s = x0 + L0*(x1 + L1*x2)``; columns are sorted within a row.
    """
    L0, L1, L2 = (int(L) for L in dims)
    n = L0 * L1 * L2
    rng = np.random.default_rng(seed)
    diag = 6.0 + rng.uniform(diag_lo, diag_hi, size=n)
    s = np.arange(n, dtype=np.int64)
    c = np.stack([s % L0, (s // L0) % L1, s // (L0 * L1)], axis=1)
    strides = (1, L0, L0 * L1)
    ext = (L0, L1, L2)
    cols = [s[:, None]]
    vals = [diag[:, None].astype(np.complex128)]
    valid = [np.ones((n, 1), dtype=bool)]
    for mu in range(3):
        for step in (-1, +1):
            ok = (c[:, mu] + step >= 0) & (c[:, mu] + step < ext[mu])
            cols.append((s + step * strides[mu])[:, None])
            vals.append(np.full((n, 1), -1.0 + 0j))
            valid.append(ok[:, None])
    cols = np.concatenate(cols, axis=1)
    vals = np.concatenate(vals, axis=1)
    valid = np.concatenate(valid, axis=1)
    cols = np.where(valid, cols, np.iinfo(np.int64).max)
    order = np.argsort(cols, axis=1, kind="stable")
    cols = np.take_along_axis(cols, order, axis=1)
    vals = np.take_along_axis(vals, order, axis=1)
    valid = np.take_along_axis(valid, order, axis=1)
    counts = valid.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    return rowptr, cols[valid].astype(np.int32), np.ascontiguousarray(vals[valid])


def poisson5pt_csr(nx: int, ny: int):
    """2-D 5-point Poisson matrix on an nx x ny grid with Dirichlet boundaries: 4 on the
    diagonal and -1 for each in-grid neighbour (the matrix of the paper's benchmark, a
    1000 x 1000 grid there).  Sites are numbered ``s = x + nx*y``; columns sorted within a
    row; stored as complex128 with zero imaginary part (real symmetric positive definite,
    given to the solver directly as A)."""
    nx, ny = int(nx), int(ny)
    n = nx * ny
    s = np.arange(n, dtype=np.int64)
    x, y = s % nx, s // nx
    # neighbours in column order: below (y-1), left (x-1), self, right (x+1), above (y+1)
    cand = [(s - nx, y > 0, -1.0), (s - 1, x > 0, -1.0), (s, np.ones(n, bool), 4.0),
            (s + 1, x < nx - 1, -1.0), (s + nx, y < ny - 1, -1.0)]
    cols = np.stack([c for c, _, _ in cand], axis=1)
    valid = np.stack([v for _, v, _ in cand], axis=1)
    vals = np.broadcast_to(np.array([v for _, _, v in cand], dtype=np.complex128), cols.shape)
    counts = valid.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    return rowptr, cols[valid].astype(np.int32), np.ascontiguousarray(vals[valid])


def random_sparse_csr(n: int, per_row: int, seed: int, diag: complex = 0.0, empty_rows=()):
    """Random complex sparse matrix with ``per_row`` distinct sorted columns per row.

    The matrix is in general not normal, so M^H M and M M^H differ; ``diag`` is added on
    the diagonal (as an extra entry when the random pattern misses it).  Rows listed in
    ``empty_rows`` hold no entry at all.
    """
    rng = np.random.default_rng(seed)
    per_row = min(int(per_row), int(n))
    empty = set(int(i) for i in empty_rows)
    rowptr = [0]
    cols, vals = [], []
    for i in range(int(n)):
        if i in empty:
            rowptr.append(rowptr[-1])
            continue
        c = rng.choice(n, size=per_row, replace=False)
        g = rng.standard_normal((per_row, 2))
        v = (g[:, 0] + 1j * g[:, 1]) / np.sqrt(2.0)
        if diag != 0.0:
            if i in c:
                v[np.nonzero(c == i)[0][0]] += diag
            else:
                c = np.append(c, i)
                v = np.append(v, diag)
        o = np.argsort(c)
        cols.append(c[o])
        vals.append(v[o])
        rowptr.append(rowptr[-1] + c.size)
    col = np.concatenate(cols).astype(np.int32) if cols else np.zeros(0, np.int32)
    val = np.concatenate(vals).astype(np.complex128) if vals else np.zeros(0, np.complex128)
    return np.asarray(rowptr, dtype=np.int64), col, val
