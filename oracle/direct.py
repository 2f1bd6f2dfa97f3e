"""The plain definition of the result, x_k = (A + sigma_k I)^{-1} b (Section 2,
eq. linprob), computed without any Krylov method.  Test infrastructure only.

* ``dense_solve``      -- LAPACK solve of the dense shifted matrix (small lattices).
* ``free_field_solve`` -- closed form for unit links: the staggered D satisfies
  -D^2 = (1/4) sum_mu (2 - T_mu^2 - T_mu^-2) with T_mu the unit shift (the staggered
  phases cancel in D^2), so A = m^2 - D^2 is diagonal in the Fourier basis of every
  colour with eigenvalue m^2 + sum_mu sin^2(2 pi n_mu / L_mu).
* ``pure_gauge_solve`` -- for links U_mu(x) = g(x) g(x+mu)^H the operator is
  M = G M_free G^H with G = diag(g(x)), hence x_k = G x_k^free(G^H b).
"""
from __future__ import annotations

import numpy as np

from .operators import csr_matrix_of


def dense_from_csr(rowptr, col, vals, n) -> np.ndarray:
    return csr_matrix_of(rowptr, col, vals, n).toarray()


def dense_solve(kind, rowptr, col, vals, n, b, sigma) -> np.ndarray:
    """x_k = (A + sigma_k I)^{-1} b for every shift, dense FP64; returns (ns, n)."""
    m = dense_from_csr(rowptr, col, vals, n)
    a = m.conj().T @ m if kind == "mhm" else m  # "herm" and "general": A as given
    eye = np.eye(int(n))
    b = np.asarray(b, dtype=np.complex128)
    return np.stack([np.linalg.solve(a + float(sk) * eye, b) for sk in np.ravel(sigma)])


def free_field_eigenvalues(dims, mass) -> np.ndarray:
    """m^2 + sum_mu sin^2(p_mu) on the FFT grid of shape (L3, L2, L1, L0)."""
    L0, L1, L2, L3 = (int(L) for L in dims)
    grids = np.meshgrid(2 * np.pi * np.arange(L3) / L3, 2 * np.pi * np.arange(L2) / L2,
                        2 * np.pi * np.arange(L1) / L1, 2 * np.pi * np.arange(L0) / L0,
                        indexing="ij")
    return mass * mass + sum(np.sin(g) ** 2 for g in grids)


def free_field_solve(dims, mass, b, sigma) -> np.ndarray:
    """Fourier closed form of (A + sigma_k)^{-1} b for unit links; returns (ns, n)."""
    L0, L1, L2, L3 = (int(L) for L in dims)
    lam = free_field_eigenvalues(dims, mass)
    # vector index 3*s + c with s = x0 + L0*(x1 + L1*(x2 + L2*x3)) -> (L3, L2, L1, L0, 3)
    bf = np.fft.fftn(np.asarray(b, dtype=np.complex128).reshape(L3, L2, L1, L0, 3),
                     axes=(0, 1, 2, 3))
    out = []
    for sk in np.ravel(sigma):
        xf = bf / (lam + float(sk))[..., None]
        out.append(np.fft.ifftn(xf, axes=(0, 1, 2, 3)).reshape(-1))
    return np.stack(out)


def pure_gauge_solve(dims, mass, g, b, sigma) -> np.ndarray:
    """Closed form for pure-gauge links U_mu(x) = g(x) g(x+mu)^H; returns (ns, n)."""
    v = g.shape[0]
    b3 = np.asarray(b, dtype=np.complex128).reshape(v, 3)
    gh_b = np.einsum("sba,sb->sa", np.conj(g), b3).reshape(-1)     # G^H b
    xfree = free_field_solve(dims, mass, gh_b, sigma)
    out = []
    for xk in xfree:
        out.append(np.einsum("sab,sb->sa", g, xk.reshape(v, 3)).reshape(-1))  # G x
    return np.stack(out)
