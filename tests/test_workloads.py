"""Pins of the synthetic inputs against facts of the mathematics (no GPU)."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle.direct import free_field_eigenvalues


def _csr(rowptr, col, vals, n):
    return sp.csr_matrix((vals, col.astype(np.int64), rowptr), shape=(n, n))


def test_haar_su3_is_special_unitary():
    u = W.haar_su3(np.random.default_rng(7), 500)
    eye = np.eye(3)
    assert np.abs(np.einsum("kba,kbc->kac", u.conj(), u) - eye).max() < 1e-14
    assert np.abs(np.linalg.det(u) - 1.0).max() < 1e-14


def test_haar_su3_is_not_degenerate():
    # Haar measure: E[|U_ab|^2] = 1/3 for every entry, E[U_ab] = 0
    u = W.haar_su3(np.random.default_rng(11), 20000)
    assert np.abs(np.mean(np.abs(u) ** 2, axis=0) - 1.0 / 3.0).max() < 0.01
    assert np.abs(np.mean(u, axis=0)).max() < 0.02


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (3, 4, 5, 6)])
def test_staggered_structure(dims):
    links = W.random_su3_links(dims, 5)
    rowptr, col, vals = W.staggered_csr(links, dims, 0.1)
    n = 3 * W.lattice_volume(dims)
    assert rowptr.dtype == np.int64 and col.dtype == np.int32 and vals.dtype == np.complex128
    assert rowptr.size == n + 1 and np.all(np.diff(rowptr) == 25)
    c = col.reshape(n, 25)
    assert np.all(np.diff(c, axis=1) > 0), "columns sorted and distinct"
    assert c.min() >= 0 and c.max() < n
    m = _csr(rowptr, col, vals, n)
    d = m - 0.1 * sp.eye(n)
    # D is exactly anti-Hermitian: D^H = -D, entry by entry
    assert abs(d + d.conj().T).max() == 0.0
    # diagonal holds exactly the mass
    assert np.all(m.diagonal() == 0.1)


def test_staggered_eta_convention():
    dims = (4, 4, 4, 4)
    eta = W.staggered_eta(dims)
    c = W.site_coords(dims)
    assert np.all(eta[0] == 1)
    assert np.all(eta[1] == (-1.0) ** c[:, 0])
    assert np.all(eta[2] == (-1.0) ** (c[:, 0] + c[:, 1]))
    assert np.all(eta[3] == (-1.0) ** (c[:, 0] + c[:, 1] + c[:, 2]))
    # site numbering: x0 fastest
    assert tuple(c[1]) == (1, 0, 0, 0) and tuple(c[4]) == (0, 1, 0, 0)
    assert tuple(c[64]) == (0, 0, 0, 1)


def test_normal_operator_spectrum_bounds():
    dims = (4, 4, 4, 4)
    rowptr, col, vals = W.staggered_csr(W.random_su3_links(dims, 1000), dims, 0.1)
    m = _csr(rowptr, col, vals, 768).toarray()
    a = m.conj().T @ m
    assert np.abs(a - a.conj().T).max() < 1e-15
    ev = np.linalg.eigvalsh(a)
    assert ev.min() >= 0.01 * (1 - 1e-12)
    # A = m^2 - D^2 exactly as matrices
    d = m - 0.1 * np.eye(768)
    assert np.abs(a - (0.01 * np.eye(768) - d @ d)).max() < 1e-13


def test_free_field_spectrum():
    dims = (4, 4, 4, 6)
    rowptr, col, vals = W.staggered_csr(W.free_links(dims), dims, 0.3)
    n = 3 * W.lattice_volume(dims)
    m = _csr(rowptr, col, vals, n).toarray()
    ev = np.linalg.eigvalsh(m.conj().T @ m)
    lam = np.repeat(free_field_eigenvalues(dims, 0.3).ravel(), 3)
    assert np.abs(np.sort(ev) - np.sort(lam)).max() < 1e-13


def test_gauge_covariance():
    dims = (4, 4, 4, 4)
    links = W.random_su3_links(dims, 21)
    g = W.haar_su3(np.random.default_rng(22), W.lattice_volume(dims))
    lt = np.empty_like(links)
    for mu in range(4):
        fwd = W.neighbour(dims, mu, +1)
        lt[mu] = g @ links[mu] @ np.conj(np.swapaxes(g[fwd], 1, 2))
    n = 768
    m = _csr(*W.staggered_csr(links, dims, 0.2), n)
    mt = _csr(*W.staggered_csr(lt, dims, 0.2), n)
    gb = sp.block_diag(list(g), format="csr")
    assert abs(mt - gb @ m @ gb.conj().T).max() < 1e-14


def test_pure_gauge_links_are_gauge_transform_of_unit():
    dims = (4, 4, 4, 4)
    links, g = W.pure_gauge_links(dims, 3)
    n = 768
    m = _csr(*W.staggered_csr(links, dims, 0.2), n)
    m0 = _csr(*W.staggered_csr(W.free_links(dims), dims, 0.2), n)
    gb = sp.block_diag(list(g), format="csr")
    assert abs(m - gb @ m0 @ gb.conj().T).max() < 1e-14


def test_laplacian7():
    rowptr, col, vals = W.laplacian7_csr((32, 32, 32), 1)
    assert col.size == 223232
    n = 32 ** 3
    a = _csr(rowptr, col, vals, n)
    assert abs(a - a.T).max() == 0.0 and np.all(vals.imag == 0)
    d = a.diagonal().real
    assert d.min() >= 6.01 and d.max() <= 7.0
    # small case: positive definite, smallest eigenvalue above min of random diagonal
    rowptr, col, vals = W.laplacian7_csr((4, 3, 5), 2)
    a = _csr(rowptr, col, vals, 60).toarray().real
    ev = np.linalg.eigvalsh(a)
    assert ev.min() > 0.01
    for i in range(60):
        assert np.all(np.diff(col[rowptr[i]:rowptr[i + 1]]) > 0)


def test_poisson5pt_spectrum_and_structure():
    # the 5-point Dirichlet Laplacian's eigenvalues are known in closed form:
    # 4 - 2 cos(i pi / (nx+1)) - 2 cos(j pi / (ny+1)), i = 1..nx, j = 1..ny
    nx, ny = 7, 5
    rowptr, col, vals = W.poisson5pt_csr(nx, ny)
    n = nx * ny
    assert col.size == 5 * n - 2 * (nx + ny)
    a = _csr(rowptr, col, vals, n).toarray()
    assert np.all(a.imag == 0) and np.array_equal(a, a.T)
    i = np.arange(1, nx + 1)[:, None]
    j = np.arange(1, ny + 1)[None, :]
    closed = np.sort((4 - 2 * np.cos(i * np.pi / (nx + 1)) - 2 * np.cos(j * np.pi / (ny + 1))).ravel())
    assert np.allclose(np.linalg.eigvalsh(a.real), closed, rtol=0, atol=1e-12)
    for r in range(n):
        assert np.all(np.diff(col[rowptr[r]:rowptr[r + 1]]) > 0)
    # the paper's size: 10^6 rows, 4,996,000 entries
    rowptr, col, vals = W.poisson5pt_csr(1000, 1000)
    assert rowptr[-1] == col.size == 5 * 10**6 - 4000


def test_random_sparse_is_not_normal():
    rowptr, col, vals = W.random_sparse_csr(50, 4, 3, diag=3.0)
    m = _csr(rowptr, col, vals, 50).toarray()
    assert np.abs(m.conj().T @ m - m @ m.conj().T).max() > 0.1


def test_shifts_and_rhs():
    s = W.logspace_shifts(1e-4, 1.0, 8)
    assert s[0] == pytest.approx(1e-4) and s[-1] == pytest.approx(1.0) and s.size == 8
    assert np.allclose(np.diff(np.log10(s)), 4.0 / 7.0)
    b = W.gaussian_rhs(200000, 3)
    assert abs(np.mean(np.abs(b) ** 2) - 1.0) < 0.01
    assert np.array_equal(W.gaussian_rhs(10, 9), W.gaussian_rhs(10, 9))


def test_config_sizes():
    c0 = W.make_config("c0")
    assert c0["n"] == 768 and c0["vals"].size == 19200 and c0["sigma"].size == 8
    c3 = W.make_config("c3")
    assert c3["n"] == 12288 and c3["vals"].size == 307200 and c3["c"].size == 10
    assert c3["fd_nz"].size == 32
