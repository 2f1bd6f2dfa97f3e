"""GPU: every shift at full size against the oracle, element by element.

* 16^4 (n = 196,608, 12 shifts): every shift's solution against the FP64 oracle CG-M
  (FP64 path: same tolerance, iterations and freeze iterations within +-2; mixed path:
  tol 1e-12 against the oracle at 1e-13, since ||dx||/||x|| <= kappa_k rho_k);
* 32^3 x 64 (n = 6,291,456, 16 shifts): pure-gauge links U_mu(x) = g(x) g(x+mu)^H make
  M = G M_free G^H, whose inverse the oracle writes in closed form with FFTs; every
  shift of the FP64 and of the mixed solve against it at tol 1e-12;
* the 64-system batch: every right-hand side of two systems of each lattice size and of
  two Laplacians against the oracle CG-M.

Solution parity: Section 2, eq. linprob (x_k = (A + sigma_k)^{-1} b).
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.linalg.norm(a - b, axis=-1) / np.linalg.norm(b, axis=-1)


def _op(p, cuda, kind="mhm"):
    from paper_1102_2143_amd import Operator
    return Operator(p["rowptr"], p["col"], p["vals"], p["n"], kind=kind, device=cuda)


# ---- 16^4 -------------------------------------------------------------------------------

@pytest.fixture(scope="module")
def c1():
    p = W.make_config("c1")
    p["apply"] = O.shifted_apply("mhm", p["rowptr"], p["col"], p["vals"], p["n"])
    p["oracle"] = {}
    return p


def _c1_oracle(c1, tol):
    if tol not in c1["oracle"]:
        print(f"[gpu] c1 oracle CG-M at tol {tol:g}", flush=True)
        c1["oracle"][tol] = O.cg_m(c1["apply"], c1["b"], c1["sigma"], tol=tol)
    return c1["oracle"][tol]


@pytest.mark.timeout(900)
def test_c1_fp64_every_shift_matches_oracle(c1, cuda):
    print("[gpu] c1 16^4 fp64: every shift vs oracle", flush=True)
    op = _op(c1, cuda)
    op.set_shifts(c1["sigma"])
    x, info = op.solve(c1["b"], tol=1e-10, prec="fp64")
    ref = _c1_oracle(c1, 1e-10)
    err = _rel(x.cpu().numpy(), ref["x"])
    print(f"[gpu] c1 fp64 iters gpu={info['iters']} oracle={ref['iters']} "
          f"max err={err.max():.3e}", flush=True)
    assert info["status"] == "ok"
    assert np.all(info["true_rel_res"] <= 1e-10)
    assert np.all(err <= 1e-8), err
    assert abs(info["iters"] - ref["iters"]) <= 2
    assert np.all(np.abs(info["freeze_iter"] - ref["freeze_iter"]) <= 2)
    op.close()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_c1_stencil_every_shift_matches_oracle(c1, cuda, prec):
    # the matrix-free operator built from the same links as the recipe's CSR
    from paper_1102_2143_amd import Operator
    cfg = W.CONFIGS["c1"]
    print(f"[gpu] c1 16^4 stencil {prec}: every shift vs oracle", flush=True)
    links = W.random_su3_links(cfg["dims"], cfg["seed_links"])
    op = Operator.staggered(links, cfg["dims"], cfg["mass"], device=cuda)
    op.set_shifts(c1["sigma"])
    tol, otol = (1e-10, 1e-10) if prec == "fp64" else (1e-12, 1e-13)
    x, info = op.solve(c1["b"], tol=tol, prec=prec, format="stencil")
    ref = _c1_oracle(c1, otol)
    err = _rel(x.cpu().numpy(), ref["x"])
    print(f"[gpu] c1 stencil {prec} iters gpu={info['iters']} oracle={ref['iters']} "
          f"max err={err.max():.3e}", flush=True)
    assert info["status"] == "ok"
    assert np.all(info["true_rel_res"] <= tol)
    assert np.all(err <= 1e-8), err
    if prec == "fp64":
        assert abs(info["iters"] - ref["iters"]) <= 2
        assert np.all(np.abs(info["freeze_iter"] - ref["freeze_iter"]) <= 2)
    op.close()


@pytest.mark.timeout(900)
def test_c1_mixed_every_shift_matches_tightened_oracle(c1, cuda):
    print("[gpu] c1 16^4 mixed at 1e-12: every shift vs oracle at 1e-13", flush=True)
    op = _op(c1, cuda)
    op.set_shifts(c1["sigma"])
    x, info = op.solve(c1["b"], tol=1e-12, prec="mixed")
    ref = _c1_oracle(c1, 1e-13)
    err = _rel(x.cpu().numpy(), ref["x"])
    print(f"[gpu] c1 mixed iters gpu={info['iters']} oracle={ref['iters']} "
          f"max err={err.max():.3e} max res={info['true_rel_res'].max():.2e}", flush=True)
    assert info["status"] == "ok"
    assert np.all(info["true_rel_res"] <= 1e-12)
    assert np.all(err <= 1e-8), err
    op.close()


# ---- 32^3 x 64, pure gauge --------------------------------------------------------------

@pytest.fixture(scope="module")
def c2_pure_gauge():
    cfg = W.CONFIGS["c2"]
    dims, mass = cfg["dims"], cfg["mass"]
    print("[gpu] c2 pure-gauge problem and FFT closed form", flush=True)
    links, g = W.pure_gauge_links(dims, cfg["seed_links"])
    rowptr, col, vals = W.staggered_csr(links, dims, mass)
    n = 3 * W.lattice_volume(dims)
    b = W.gaussian_rhs(n, cfg["seed_b"])
    sigma = W.logspace_shifts(*cfg["shifts"])
    xs = O.pure_gauge_solve(dims, mass, g, b, sigma)
    # spectrum of A = M^H M is that of the free field: [m^2, m^2 + 4]
    kappa = (mass ** 2 + 4.0 + sigma) / (mass ** 2 + sigma)
    return dict(n=n, rowptr=rowptr, col=col, vals=vals, b=b, sigma=sigma, x=xs, kappa=kappa,
                links=links, dims=dims, mass=mass)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec,fmt", [("fp64", "sell"), ("mixed", "sell"), ("fp64", "stencil"),
                                      ("mixed", "stencil")])
def test_c2_pure_gauge_every_shift_matches_closed_form(c2_pure_gauge, cuda, prec, fmt):
    p = c2_pure_gauge
    print(f"[gpu] c2 32^3x64 pure gauge {prec} {fmt} at 1e-12: every shift vs FFT", flush=True)
    if fmt == "stencil":
        from paper_1102_2143_amd import Operator
        op = Operator.staggered(p["links"], p["dims"], p["mass"], device=cuda)
    else:
        op = _op(p, cuda)
    op.set_shifts(p["sigma"])
    x, info = op.solve(p["b"], tol=1e-12, prec=prec, format=fmt)
    assert info["status"] == "ok", info["status"]
    rho = info["true_rel_res"]
    err = np.array([_rel(x[k].cpu().numpy(), p["x"][k]) for k in range(p["sigma"].size)])
    for k in range(p["sigma"].size):
        print(f"[gpu] c2 pg {prec} sigma={p['sigma'][k]:.1e} err={err[k]:.2e} "
              f"rho={rho[k]:.2e} kappa*rho={p['kappa'][k] * rho[k]:.2e}", flush=True)
    assert np.all(rho <= 1e-12)
    # the error bound ||dx||/||x|| <= kappa_k rho_k, and the spec bar
    assert np.all(err <= p["kappa"] * rho * 1.01 + 1e-14)
    assert np.all(err <= 1e-8)
    op.close()


# ---- the 64-system batch ----------------------------------------------------------------

def _sampled_systems(systems):
    """Indices of two systems of each staggered lattice size and two Laplacians."""
    picked, seen = [], {}
    for i, p in enumerate(systems):
        key = (p["kind"], tuple(p["dims"]))
        if seen.get(key, 0) < 2:
            seen[key] = seen.get(key, 0) + 1
            picked.append(i)
    return picked


@pytest.fixture(scope="module")
def c4():
    systems = W.make_config("c4")["systems"]
    return dict(systems=systems, picked=_sampled_systems(systems), oracle={})


def _c4_oracle(c4, i, q, tol):
    key = (i, q, tol)
    if key not in c4["oracle"]:
        p = c4["systems"][i]
        ap = O.shifted_apply(p["kind"], p["rowptr"], p["col"], p["vals"], p["n"])
        c4["oracle"][key] = O.cg_m(ap, np.atleast_2d(p["b"])[q], p["sigma"], tol=tol)
    return c4["oracle"][key]


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec,tol,otol", [("fp64", 1e-10, 1e-10), ("mixed", 1e-12, 1e-13)])
def test_c4_batch_sampled_systems_match_oracle(c4, cuda, prec, tol, otol):
    from paper_1102_2143_amd import Operator, solve_batched
    systems = c4["systems"]
    print(f"[gpu] c4 64-system batch {prec} at {tol:g}: sampled systems vs oracle", flush=True)
    ops = []
    for p in systems:
        op = Operator(p["rowptr"], p["col"], p["vals"], p["n"], kind=p["kind"], device=cuda)
        op.set_shifts(p["sigma"])
        ops.append(op)
    xs, infos, status = solve_batched(ops, [p["b"] for p in systems], tol=tol, prec=prec)
    assert status == "ok"
    first = np.cumsum([0] + [np.atleast_2d(p["b"]).shape[0] for p in systems])
    worst = 0.0
    for i in c4["picked"]:
        p = systems[i]
        for q in range(np.atleast_2d(p["b"]).shape[0]):
            ref = _c4_oracle(c4, i, q, otol)
            info = infos[first[i] + q]
            err = _rel(xs[i][q].cpu().numpy(), ref["x"])
            worst = max(worst, float(err.max()))
            assert np.all(info["true_rel_res"] <= tol), (i, q, info["true_rel_res"])
            assert np.all(err <= 1e-8), (i, q, err)
            if prec == "fp64":
                assert abs(info["iters"] - ref["iters"]) <= 2, (i, q, info["iters"], ref["iters"])
    print(f"[gpu] c4 {prec}: {len(c4['picked'])} systems x 4 rhs, max err {worst:.2e}", flush=True)
    for op in ops:
        op.close()
