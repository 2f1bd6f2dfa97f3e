"""GPU: the matrix-free staggered operator (msc_op_create_staggered) against the oracle.

The operator is built from the gauge links; its iteration applies M = m + D and
M^H = m - D from them (Section 3: a custom linear operator kernel in place of the
stored matrix), while the library also builds the equivalent CSR for its other kernels.

* the CSR it builds on the device equals the one the input generator writes on the host
  (the products through it agree bit for bit), on cubic and non-cubic lattices with the
  smallest extent 3;
* the 4^4 solve through the links against the oracle CG-M (FP64: per-shift error
  <= 1e-8, iterations and freeze iterations within 2; mixed at 1e-12 against the oracle
  at 1e-13), and against the dense solve;
* new links through msc_op_update_links give what a fresh operator gives;
* SU(3) links are read as their first two rows (the third rebuilt in the kernels):
  reported by storage(), and links off SU(3) (scaled, or a U(3) phase) keep all nine
  values, through creation and through update_links, with the same parity;
* the misuse cases are rejected;
* the site kernels on lattices whose volume leaves a partial block of 64 sites, on one
  whose blocks follow the lattice order, and with nine-value links in both phases of a
  mixed solve, against the oracle;
* the heads and K2 marching along t (columns of 16, 8 or 4 t-slices, runs that start
  inside a column, columns shared by several waves, grids with and without the per-XCD
  split; the FP64 head with its recurrence t' = M r + b t, the complex64 head gathering
  p') against the oracle.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.linalg.norm(a - b, axis=-1) / np.linalg.norm(b, axis=-1)


def _pair(dims, mass, seed, cuda):
    from paper_1102_2143_amd import Operator
    links = W.random_su3_links(dims, seed)
    rowptr, col, vals = W.staggered_csr(links, dims, mass)
    n = 3 * W.lattice_volume(dims)
    st = Operator.staggered(links, dims, mass, device=cuda)
    cs = Operator(rowptr, col, vals, n, kind="mhm", device=cuda)
    return dict(links=links, rowptr=rowptr, col=col, vals=vals, n=n, st=st, cs=cs)


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (3, 4, 5, 6), (6, 3, 4, 8)])
def test_device_csr_equals_host_csr(cuda, dims):
    print(f"[gpu] stencil csr dims={dims}", flush=True)
    p = _pair(dims, 0.07, 91, cuda)
    v = W.gaussian_rhs(p["n"], 5)
    for prec in ("fp64", "mixed"):
        for shift in (0.0, 0.3):
            a = p["st"].apply(v, shift=shift, prec=prec)
            b = p["cs"].apply(v, shift=shift, prec=prec)
            assert bool((a == b).all()), (dims, prec, shift)
    # and both equal the oracle's product to rounding
    ref = O.shifted_apply("mhm", p["rowptr"], p["col"], p["vals"], p["n"])(v, 0.3)
    assert _rel(p["st"].apply(v, shift=0.3).cpu().numpy(), ref) <= 1e-14
    p["st"].close()
    p["cs"].close()


@pytest.fixture(scope="module")
def c0():
    p = W.make_config("c0")
    dims = W.CONFIGS["c0"]["dims"]
    p["links"] = W.random_su3_links(dims, W.CONFIGS["c0"]["seed_links"])
    p["dims"] = dims
    p["mass"] = W.CONFIGS["c0"]["mass"]
    p["apply"] = O.shifted_apply("mhm", p["rowptr"], p["col"], p["vals"], p["n"])
    p["ref"] = O.cg_m(p["apply"], p["b"], p["sigma"], tol=1e-10)
    return p


def test_c0_links_match_the_input_csr(c0):
    # the recipe's links reproduce the recipe's CSR exactly (the stencil tests below
    # compare the link-built operator with the oracle on that CSR)
    rowptr, col, vals = W.staggered_csr(c0["links"], c0["dims"], c0["mass"])
    assert np.array_equal(col, c0["col"]) and np.array_equal(vals, c0["vals"])


def test_c0_fp64_matches_oracle(c0, cuda):
    from paper_1102_2143_amd import Operator
    print("[gpu] stencil c0 fp64 vs oracle", flush=True)
    op = Operator.staggered(c0["links"], c0["dims"], c0["mass"], device=cuda)
    op.set_shifts(c0["sigma"])
    x, info = op.solve(c0["b"], tol=1e-10, prec="fp64", format="stencil")
    ref = c0["ref"]
    assert info["status"] == "ok"
    assert np.all(_rel(x.cpu().numpy(), ref["x"]) <= 1e-8)
    assert abs(info["iters"] - ref["iters"]) <= 2
    assert np.all(np.abs(info["freeze_iter"] - ref["freeze_iter"]) <= 2)
    assert np.all(info["true_rel_res"] <= 1e-10)
    dense = O.dense_solve("mhm", c0["rowptr"], c0["col"], c0["vals"], c0["n"], c0["b"], c0["sigma"])
    assert np.all(_rel(x.cpu().numpy(), dense) <= 1e-8)
    # format auto takes the links for this operator: the same bits
    x2, info2 = op.solve(c0["b"], tol=1e-10, prec="fp64")
    assert info2["iters"] == info["iters"] and bool((x2 == x).all())
    op.close()


def test_c0_mixed_matches_tightened_oracle(c0, cuda):
    from paper_1102_2143_amd import Operator
    print("[gpu] stencil c0 mixed at 1e-12 vs oracle at 1e-13", flush=True)
    op = Operator.staggered(c0["links"], c0["dims"], c0["mass"], device=cuda)
    op.set_shifts(c0["sigma"])
    x, info = op.solve(c0["b"], tol=1e-12, prec="mixed")
    ref = O.cg_m(c0["apply"], c0["b"], c0["sigma"], tol=1e-13)
    assert info["status"] == "ok"
    assert info["n_reliable"] > 0
    assert np.all(info["true_rel_res"] <= 1e-12)
    assert np.all(_rel(x.cpu().numpy(), ref["x"]) <= 1e-8)
    op.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_stencil_and_stored_matrix_agree(c0, cuda, prec):
    # the same operator read from links and from the sliced ELLPACK copy: the products
    # differ only in summation order, so the solutions agree to the solve's accuracy
    from paper_1102_2143_amd import Operator
    op = Operator.staggered(c0["links"], c0["dims"], c0["mass"], device=cuda)
    op.set_shifts(c0["sigma"])
    xs, i_s = op.solve(c0["b"], tol=1e-12, prec=prec, format="stencil")
    xm, i_m = op.solve(c0["b"], tol=1e-12, prec=prec, format="sell")
    assert abs(i_s["iters"] - i_m["iters"]) <= 2
    assert np.all(_rel(xs.cpu().numpy(), xm.cpu().numpy()) <= 1e-8)
    op.close()


def test_update_links_matches_a_fresh_operator(c0, cuda):
    from paper_1102_2143_amd import Operator
    dims, mass = c0["dims"], c0["mass"]
    op = Operator.staggered(c0["links"], dims, mass, device=cuda)
    op.set_shifts(c0["sigma"])
    new = W.random_su3_links(dims, 4242)
    op.update_links(new)
    x1, i1 = op.solve(c0["b"], tol=1e-10, prec="fp64")
    fresh = Operator.staggered(new, dims, mass, device=cuda)
    fresh.set_shifts(c0["sigma"])
    x2, i2 = fresh.solve(c0["b"], tol=1e-10, prec="fp64")
    assert i1["iters"] == i2["iters"] and bool((x1 == x2).all())
    rowptr, col, vals = W.staggered_csr(new, dims, mass)
    ref = O.cg_m(O.shifted_apply("mhm", rowptr, col, vals, c0["n"]), c0["b"], c0["sigma"], tol=1e-10)
    assert np.all(_rel(x1.cpu().numpy(), ref["x"]) <= 1e-8)
    op.close()
    fresh.close()


def test_misuse_is_rejected(c0, cuda):
    from paper_1102_2143_amd import MscError, Operator
    op = Operator.staggered(c0["links"], c0["dims"], c0["mass"], device=cuda)
    with pytest.raises(MscError):
        op.update_values(c0["vals"])
    cs = Operator(c0["rowptr"], c0["col"], c0["vals"], c0["n"], kind="mhm", device=cuda)
    cs.set_shifts(c0["sigma"])
    with pytest.raises(MscError):
        cs.solve(c0["b"], format="stencil")
    with pytest.raises(MscError):
        cs.update_links(c0["links"])
    op.close()
    cs.close()


def test_two_row_links_and_their_fallback(c0, cuda):
    from paper_1102_2143_amd import Operator
    dims, mass = c0["dims"], c0["mass"]
    op = Operator.staggered(c0["links"], dims, mass, device=cuda)
    assert op.storage()["two_rows"] is True
    op.set_shifts(c0["sigma"])
    for prec in ("fp64", "mixed"):
        x, info = op.solve(c0["b"], tol=1e-10, prec=prec)
        assert info["status"] == "ok" and np.all(info["true_rel_res"] <= 1e-10)
        assert np.all(_rel(x.cpu().numpy(), c0["ref"]["x"]) <= 1e-8)
        if prec == "fp64":
            assert abs(info["iters"] - c0["ref"]["iters"]) <= 2
    # links off SU(3): a U(3) phase on one link, then every link scaled
    for bad in ("phase", "scale"):
        links = np.array(c0["links"], copy=True)
        if bad == "phase":
            links[2, 5] = links[2, 5] * np.exp(0.3j)
        else:
            links = links * 1.01
        op.update_links(links)
        assert op.storage()["two_rows"] is False
        rowptr, col, vals = W.staggered_csr(links, dims, mass)
        ap = O.shifted_apply("mhm", rowptr, col, vals, c0["n"])
        ref = O.cg_m(ap, c0["b"], c0["sigma"], tol=1e-10)
        x, info = op.solve(c0["b"], tol=1e-10, prec="fp64")
        assert info["status"] == "ok"
        assert np.all(_rel(x.cpu().numpy(), ref["x"]) <= 1e-8)
        assert abs(info["iters"] - ref["iters"]) <= 2
        fresh = Operator.staggered(links, dims, mass, device=cuda)
        assert fresh.storage()["two_rows"] is False
        fresh.close()
    # back to SU(3) links: two rows again
    op.update_links(c0["links"])
    assert op.storage()["two_rows"] is True
    op.close()


@pytest.mark.parametrize("dims", [(3, 4, 5, 6), (5, 5, 5, 7), (8, 8, 8, 8)])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_site_kernels_on_ragged_and_ordered_lattices(cuda, dims, prec):
    # the iteration's kernels take blocks of 64 sites: 360 and 875 sites leave a partial
    # last block, 8^4 (planes of exactly one block) sweeps its blocks in the lattice order;
    # FP64 at tol 1e-10 against the oracle CG-M (per shift <= 1e-8, iterations within 2),
    # mixed at 1e-12 against the oracle at 1e-13
    from paper_1102_2143_amd import Operator
    print(f"[gpu] stencil site kernels dims={dims} {prec}", flush=True)
    mass = 0.1
    links = W.random_su3_links(dims, 77)
    rowptr, col, vals = W.staggered_csr(links, dims, mass)
    n = 3 * W.lattice_volume(dims)
    sigma = W.logspace_shifts(1e-4, 1.0, 6)
    b = W.gaussian_rhs(n, 78)
    ap = O.shifted_apply("mhm", rowptr, col, vals, n)
    op = Operator.staggered(links, dims, mass, device=cuda)
    assert op.storage()["two_rows"] is True
    op.set_shifts(sigma)
    if prec == "fp64":
        ref = O.cg_m(ap, b, sigma, tol=1e-10)
        x, info = op.solve(b, tol=1e-10, prec="fp64")
        assert abs(info["iters"] - ref["iters"]) <= 2
        assert np.all(info["true_rel_res"] <= 1e-10)
    else:
        ref = O.cg_m(ap, b, sigma, tol=1e-13)
        x, info = op.solve(b, tol=1e-12, prec="mixed")
        assert np.all(info["true_rel_res"] <= 1e-12)
    assert info["status"] == "ok"
    assert np.all(_rel(x.cpu().numpy(), ref["x"]) <= 1e-8)
    op.close()


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (3, 4, 5, 6)])
def test_nine_value_links_in_the_mixed_solve(cuda, dims):
    # links off SU(3) keep all nine values in both phases of a mixed solve (the complex64
    # kernels read them too): mixed at 1e-12 against the oracle at 1e-13
    from paper_1102_2143_amd import Operator
    print(f"[gpu] stencil nine-value links mixed dims={dims}", flush=True)
    mass = 0.1
    links = W.random_su3_links(dims, 79) * 1.01
    rowptr, col, vals = W.staggered_csr(links, dims, mass)
    n = 3 * W.lattice_volume(dims)
    sigma = W.logspace_shifts(1e-4, 1.0, 6)
    b = W.gaussian_rhs(n, 80)
    op = Operator.staggered(links, dims, mass, device=cuda)
    assert op.storage()["two_rows"] is False
    op.set_shifts(sigma)
    x, info = op.solve(b, tol=1e-12, prec="mixed")
    ref = O.cg_m(O.shifted_apply("mhm", rowptr, col, vals, n), b, sigma, tol=1e-13)
    assert info["status"] == "ok" and np.all(info["true_rel_res"] <= 1e-12)
    assert np.all(_rel(x.cpu().numpy(), ref["x"]) <= 1e-8)
    op.close()


@pytest.mark.parametrize("dims,grid", [((8, 8, 8, 32), 16), ((8, 8, 8, 24), 8),
                                       ((8, 8, 16, 12), 12)])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_march_along_t(cuda, dims, grid, prec):
    # with the grid capped at 16 (8, 12) workgroups, 256 (192, 192) blocks of 64 sites give
    # every wave a run of 4 (6, 4) blocks in columns of 16 (8, 4) t-slices, the largest
    # power of two up to 16 that divides L_t: runs start inside columns and cross into the
    # next one; 12 workgroups are not a multiple of the 8 XCDs, so the runs are dealt
    # without the per-XCD split.
    # FP64 at tol 1e-10 against the oracle CG-M (per shift <= 1e-8, iterations within 2),
    # mixed at 1e-12 against the oracle at 1e-13
    from paper_1102_2143_amd import Operator
    # the heads take the same columns (the grid caps them alike)
    print(f"[gpu] stencil march dims={dims} grid={grid} {prec}", flush=True)
    mass = 0.1
    links = W.random_su3_links(dims, 81)
    rowptr, col, vals = W.staggered_csr(links, dims, mass)
    n = 3 * W.lattice_volume(dims)
    sigma = W.logspace_shifts(1e-4, 1.0, 6)
    b = W.gaussian_rhs(n, 82)
    ap = O.shifted_apply("mhm", rowptr, col, vals, n)
    op = Operator.staggered(links, dims, mass, device=cuda)
    assert op.storage()["two_rows"] is True
    op.set_shifts(sigma)
    if prec == "fp64":
        ref = O.cg_m(ap, b, sigma, tol=1e-10)
        x, info = op.solve(b, tol=1e-10, prec="fp64", max_grid=grid)
        assert abs(info["iters"] - ref["iters"]) <= 2
        assert np.all(info["true_rel_res"] <= 1e-10)
    else:
        ref = O.cg_m(ap, b, sigma, tol=1e-13)
        x, info = op.solve(b, tol=1e-12, prec="mixed", max_grid=grid)
        assert np.all(info["true_rel_res"] <= 1e-12)
    assert info["status"] == "ok"
    assert np.all(_rel(x.cpu().numpy(), ref["x"]) <= 1e-8)
    op.close()
