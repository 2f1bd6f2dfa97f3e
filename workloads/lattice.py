"""Gauge links and the staggered fermion matrix M = m I + D as a scalar complex CSR.

The paper's target application is lattice gauge theory: the shifted systems come from a
rational approximation whose matrix is built from the fermion operator (Section 2,
eq. linprob).  The paper is generic and fixes no operator; the conventions below are
the reading used throughout this repository:

* sites are numbered ``s = x0 + L0*(x1 + L1*(x2 + L2*x3))``; direction 3 is time;
* a row/column index is ``3*s + colour``;
* staggered phases ``eta_0 = 1`` and ``eta_mu(x) = (-1)**(x0 + ... + x_{mu-1})``;
* all directions are periodic;
* ``D[x, y] = sum_mu eta_mu(x)/2 * (U_mu(x) delta(y, x+mu) - U_mu(x-mu)^H delta(y, x-mu))``.

``D`` is anti-Hermitian, so ``A = M^H M = m^2 - D^2`` is Hermitian positive definite with
smallest eigenvalue at least ``m^2``.  Every row holds exactly 25 entries (the mass plus
eight neighbours times three colours); columns are sorted within each row.
"""
from __future__ import annotations

import numpy as np

NDIM = 4
NCOL = 3


def lattice_volume(dims) -> int:
    v = 1
    for L in dims:
        v *= int(L)
    return v


def site_coords(dims) -> np.ndarray:
    """Coordinates (V, 4) of every site in the site numbering above."""
    dims = tuple(int(L) for L in dims)
    s = np.arange(lattice_volume(dims), dtype=np.int64)
    out = np.empty((s.size, NDIM), dtype=np.int64)
    rem = s
    for mu, L in enumerate(dims):
        out[:, mu] = rem % L
        rem = rem // L
    return out


def _site_index(coords, dims) -> np.ndarray:
    s = np.zeros(coords.shape[0], dtype=np.int64)
    stride = 1
    for mu, L in enumerate(dims):
        s += (coords[:, mu] % L) * stride
        stride *= L
    return s


def neighbour(dims, mu: int, step: int) -> np.ndarray:
    """Site index of x + step*mu_hat (periodic) for every site x."""
    dims = tuple(int(L) for L in dims)
    c = site_coords(dims)
    c[:, mu] += step
    return _site_index(c, dims)


def staggered_eta(dims) -> np.ndarray:
    """Staggered phases eta_mu(x), shape (4, V), values +-1 as float64."""
    c = site_coords(dims)
    eta = np.empty((NDIM, c.shape[0]), dtype=np.float64)
    run = np.zeros(c.shape[0], dtype=np.int64)
    for mu in range(NDIM):
        eta[mu] = np.where(run % 2 == 0, 1.0, -1.0)
        run = run + c[:, mu]
    return eta


def haar_su3(rng: np.random.Generator, count: int) -> np.ndarray:
    """``count`` Haar-random SU(3) matrices, shape (count, 3, 3), complex128.

    Recipe: Z complex Gaussian; Z = QR; Q <- Q diag(R_ii/|R_ii|) is Haar on U(3);
    dividing by the principal cube root of det(Q) lands in SU(3).
    """
    g = rng.standard_normal((count, NCOL, NCOL, 2))
    z = (g[..., 0] + 1j * g[..., 1]) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=1, axis2=2)
    ph = d / np.abs(d)
    q = q * ph[:, None, :]
    det = np.linalg.det(q)
    q = q * np.exp(-1j * np.angle(det) / 3.0)[:, None, None]
    return q


def random_su3_links(dims, seed: int) -> np.ndarray:
    """Haar-random links U_mu(x), shape (4, V, 3, 3), generated direction-major."""
    rng = np.random.default_rng(seed)
    v = lattice_volume(dims)
    return haar_su3(rng, NDIM * v).reshape(NDIM, v, NCOL, NCOL)


def free_links(dims) -> np.ndarray:
    """Unit links U_mu(x) = 1 (free field)."""
    v = lattice_volume(dims)
    u = np.zeros((NDIM, v, NCOL, NCOL), dtype=np.complex128)
    u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1.0
    return u


def pure_gauge_links(dims, seed: int):
    """Pure-gauge links U_mu(x) = g(x) g(x+mu)^H with Haar g; returns (links, g)."""
    rng = np.random.default_rng(seed)
    v = lattice_volume(dims)
    g = haar_su3(rng, v)
    u = np.empty((NDIM, v, NCOL, NCOL), dtype=np.complex128)
    for mu in range(NDIM):
        fwd = neighbour(dims, mu, +1)
        u[mu] = g @ np.conj(np.swapaxes(g[fwd], 1, 2))
    return u, g


def staggered_csr(links: np.ndarray, dims, mass: float):
    """CSR of M = m I + D for the given links.

    Returns ``(rowptr int64[n+1], col int32[nnz], vals complex128[nnz])`` with
    n = 3V and exactly 25 sorted entries per row.  Every extent must be at least 3 so
    that the forward and backward neighbours of a site are distinct.
    """
    dims = tuple(int(L) for L in dims)
    if any(L < 3 for L in dims):
        raise ValueError("every lattice extent must be >= 3")
    v = lattice_volume(dims)
    n = NCOL * v
    per_row = 1 + 2 * NDIM * NCOL
    eta = staggered_eta(dims)
    cols = np.empty((v, NCOL, per_row), dtype=np.int64)
    vals = np.empty((v, NCOL, per_row), dtype=np.complex128)
    site = np.arange(v, dtype=np.int64)
    colour = np.arange(NCOL, dtype=np.int64)
    # mass term
    cols[:, :, 0] = NCOL * site[:, None] + colour[None, :]
    vals[:, :, 0] = mass
    slot = 1
    for mu in range(NDIM):
        fwd = neighbour(dims, mu, +1)
        bwd = neighbour(dims, mu, -1)
        h = 0.5 * eta[mu][:, None, None]
        # + eta/2 * U_mu(x)[a, b] at column 3*(x+mu) + b
        cols[:, :, slot:slot + NCOL] = NCOL * fwd[:, None, None] + colour[None, None, :]
        vals[:, :, slot:slot + NCOL] = h * links[mu]
        slot += NCOL
        # - eta/2 * conj(U_mu(x-mu)[b, a]) at column 3*(x-mu) + b
        cols[:, :, slot:slot + NCOL] = NCOL * bwd[:, None, None] + colour[None, None, :]
        vals[:, :, slot:slot + NCOL] = -h * np.conj(np.swapaxes(links[mu][bwd], 1, 2))
        slot += NCOL
    cols = cols.reshape(n, per_row)
    vals = vals.reshape(n, per_row)
    order = np.argsort(cols, axis=1, kind="stable")
    cols = np.take_along_axis(cols, order, axis=1)
    vals = np.take_along_axis(vals, order, axis=1)
    rowptr = np.arange(0, (n + 1) * per_row, per_row, dtype=np.int64)
    return rowptr, cols.reshape(-1).astype(np.int32), np.ascontiguousarray(vals.reshape(-1))
