"""GPU: many independent multishift solves in one batched launch sequence, each
(system, right-hand side) against the FP64 oracle."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.linalg.norm(a - b, axis=-1) / np.linalg.norm(b, axis=-1)


def _small_batch():
    systems = []
    for i, dims in enumerate([(4, 4, 4, 4), (4, 4, 4, 6), (6, 4, 4, 4)]):
        p = W.staggered_problem(dims, 0.1, 700 + i, 800 + i, (1e-4, 1.0, 6 + 2 * i), nrhs=i + 1)
        systems.append(p)
    rowptr, col, vals = W.laplacian7_csr((7, 6, 5), 900)
    systems.append(dict(kind="herm", n=210, rowptr=rowptr, col=col, vals=vals,
                        b=W.gaussian_rhs(210, 901, 4), sigma=W.logspace_shifts(1e-4, 1.0, 10)))
    return systems


def _ops(systems, cuda):
    from paper_1102_2143_amd import Operator
    ops = []
    for p in systems:
        op = Operator(p["rowptr"], p["col"], p["vals"], p["n"], kind=p["kind"], device=cuda)
        op.set_shifts(p["sigma"])
        ops.append(op)
    return ops


@pytest.mark.parametrize("prec,fmt", [("fp64", "auto"), ("mixed", "auto"), ("fp64", "csr"),
                                      ("mixed", "csr"), ("fp64", "sell32"), ("mixed", "sell32")])
def test_small_batch_matches_oracle(cuda, prec, fmt):
    # "auto": the SpMVs read each system's sliced ELLPACK copy (16-bit column offsets);
    # "sell32": the same copy with its 32-bit columns; "csr": the CSR kernels
    print(f"[gpu] batched small {prec} {fmt}", flush=True)
    from paper_1102_2143_amd import solve_batched
    systems = _small_batch()
    ops = _ops(systems, cuda)
    xs, infos, status = solve_batched(ops, [p["b"] for p in systems], tol=1e-10, prec=prec,
                                      format=fmt)
    assert status == "ok", [i["status"] for i in infos]
    t = 0
    for s, p in enumerate(systems):
        ap = O.shifted_apply(p["kind"], p["rowptr"], p["col"], p["vals"], p["n"])
        bs = np.atleast_2d(p["b"])
        for q in range(bs.shape[0]):
            # the mixed sequence runs to mixed_margin * tol (default 0.7): its Krylov path
            # is compared with the oracle's at that tolerance
            ref = O.cg_m(ap, bs[q], p["sigma"], tol=1e-10 * (0.7 if prec == "mixed" else 1.0))
            xg = xs[s][q].cpu().numpy()
            info = infos[t]
            t += 1
            assert np.all(info["true_rel_res"] <= 1e-10), (s, q, info["true_rel_res"])
            assert np.all(_rel(xg, ref["x"]) <= 1e-8), (s, q)
            # FP64: the oracle's Krylov path to +-2; mixed: against the oracle run to the
            # same stopping rule (tol * mixed_margin), with one iteration per replacement
            # of the residual by the true one on top (each reliable update perturbs the
            # Krylov sequence, which takes about one step to absorb it)
            bar = 2 if prec == "fp64" else info["n_reliable"] + 2
            assert abs(info["iters"] - ref["iters"]) <= bar, (s, q, info["iters"], ref["iters"])
            rho = np.array([np.linalg.norm(bs[q] - ap(xg[k], sk)) for k, sk in enumerate(p["sigma"])])
            assert np.all(rho / np.linalg.norm(bs[q]) <= 1e-10)
    for op in ops:
        op.close()


@pytest.mark.parametrize("fmt", ["csr", "auto"])
def test_batch_refinement_on_fresh_operators(cuda, fmt):
    # complex64 from the first iterations and no margin: most shifts end above tol and
    # the FP64 refinement (batched CG per operator) runs, as the first use of each
    # operator's refinement buffers.  Those buffers are cleared on the batch's own stream:
    # a clearing on the null stream could land after the first refinement kernels wrote
    # them (seen under profiling as a breakdown of the Laplacian's refinement).
    print(f"[gpu] batched refinement on fresh operators {fmt}", flush=True)
    from paper_1102_2143_amd import solve_batched
    systems = _small_batch()
    ops = _ops(systems, cuda)
    kw = dict(format="csr", lanes=4) if fmt == "csr" else {}
    xs, infos, status = solve_batched(ops, [p["b"] for p in systems], tol=1e-10, prec="mixed",
                                      switch_tol=1e-2, mixed_margin=1.0, **kw)
    assert status == "ok"
    assert sum(i["n_refined"] for i in infos) > 0
    t = 0
    for s, p in enumerate(systems):
        bs = np.atleast_2d(p["b"])
        for q in range(bs.shape[0]):
            info = infos[t]
            t += 1
            assert np.all(info["true_rel_res"] <= 1e-10), (s, q)
            dense = O.dense_solve(p["kind"], p["rowptr"], p["col"], p["vals"], p["n"], bs[q],
                                  p["sigma"])
            assert np.all(_rel(xs[s][q].cpu().numpy(), dense) <= 1e-8), (s, q)
    for op in ops:
        op.close()


def test_batch_result_is_independent_of_companions(cuda):
    # each system's arithmetic depends only on its own rows: alone or with others, its
    # solution is bitwise the same
    from paper_1102_2143_amd import solve_batched
    systems = _small_batch()
    ops = _ops(systems, cuda)
    xs_all, _, st1 = solve_batched(ops, [p["b"] for p in systems], tol=1e-10, prec="fp64", lanes=8,
                                    format="sell")
    xs_one, _, st2 = solve_batched([ops[2]], [systems[2]["b"]], tol=1e-10, prec="fp64", lanes=8,
                                    format="sell")
    assert st1 == "ok" and st2 == "ok"
    assert bool((xs_all[2] == xs_one[0]).all())
    # the 32-bit and the 16-bit columns name the same entries: the same bits
    xs_w, _, st3 = solve_batched(ops, [p["b"] for p in systems], tol=1e-10, prec="fp64", lanes=8,
                                 format="sell32")
    assert st3 == "ok"
    for a, b in zip(xs_all, xs_w):
        assert bool((a == b).all())
    for op in ops:
        op.close()


@pytest.mark.parametrize("steps", [2, 4, 8])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_folded_steps_match_one_step(cuda, prec, steps):
    # the batch defers shifted updates (x_0's included) and folds up to `steps` of them (at
    # most 4) into one pass: in FP64 the driving sequences, iteration counts and freezes
    # are those of one step per iteration; in a mixed solve the reliable updates recompute
    # r from x_0, whose rounding depends on the folding, so they agree within 2; the
    # solutions agree to rounding, and fewer bytes move
    print(f"[gpu] batched {steps} folded steps {prec}", flush=True)
    from paper_1102_2143_amd import solve_batched
    systems = _small_batch()
    ops = _ops(systems, cuda)
    bs = [p["b"] for p in systems]
    x1, i1, s1 = solve_batched(ops, bs, tol=1e-10, prec=prec, update_steps=1)
    x2, i2, s2 = solve_batched(ops, bs, tol=1e-10, prec=prec, update_steps=steps)
    assert s1 == "ok" and s2 == "ok"
    for a, b in zip(i1, i2):
        if prec == "fp64":
            assert a["iters"] == b["iters"]
            assert np.array_equal(a["freeze_iter"], b["freeze_iter"])
        else:
            assert abs(a["iters"] - b["iters"]) <= 2
            assert np.all(np.abs(a["freeze_iter"] - b["freeze_iter"]) <= 2)
        assert np.all(b["true_rel_res"] <= 1e-10)
    bar = 1e-11 if prec == "fp64" else 1e-6
    for a, b in zip(x1, x2):
        assert np.all(_rel(b.cpu().numpy(), a.cpu().numpy()) <= bar)
    assert sum(i["alg_bytes"] for i in i2) < sum(i["alg_bytes"] for i in i1)
    for op in ops:
        op.close()


def test_batch_rejects_bad_input(cuda):
    from paper_1102_2143_amd import MscError, solve_batched
    systems = _small_batch()[:1]
    ops = _ops(systems, cuda)
    b5 = W.gaussian_rhs(systems[0]["n"], 1, 5)
    with pytest.raises(MscError, match="right-hand sides"):
        solve_batched(ops, [b5])
    ops[0].close()


def test_c4_full_batch(cuda):
    print("[gpu] c4 batch: 64 systems x 4 rhs x 10 shifts", flush=True)
    from paper_1102_2143_amd import solve_batched
    cfg = W.make_config("c4")
    systems = cfg["systems"]
    assert len(systems) == 64
    ops = _ops(systems, cuda)
    xs, infos, status = solve_batched(ops, [p["b"] for p in systems], tol=1e-10, prec="mixed")
    print(f"[gpu] c4 status={status} t={infos[0]['seconds']:.3f}s "
          f"max res={max(i['true_rel_res'].max() for i in infos):.3e}", flush=True)
    assert status == "ok"
    assert all(np.all(i["true_rel_res"] <= 1e-10) for i in infos)
    # independent spot checks with the oracle's operator on two systems
    for s in (0, 63):
        p = systems[s]
        ap = O.shifted_apply(p["kind"], p["rowptr"], p["col"], p["vals"], p["n"])
        xg = xs[s][1].cpu().numpy()
        rho = np.array([np.linalg.norm(p["b"][1] - ap(xg[k], sk)) for k, sk in enumerate(p["sigma"])])
        assert np.all(rho / np.linalg.norm(p["b"][1]) <= 1e-10)
    for op in ops:
        op.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_at_maximum_shifts_and_rhs(cuda, prec):
    # 16 shifts and 4 right-hand sides, the most a batched system takes (17 shifts are
    # rejected), beside a smaller system; every (system, rhs) against the oracle.  Mixed
    # runs at tol 1e-12 against the oracle at 1e-13 (solution error <= kappa * residual)
    from paper_1102_2143_amd import solve_batched, MscError
    print(f"[gpu] batched max shifts and rhs {prec}", flush=True)
    big = W.staggered_problem((4, 4, 4, 6), 0.1, 710, 810, (1e-4, 10.0, 16), nrhs=4)
    small = W.staggered_problem((4, 4, 4, 4), 0.1, 711, 811, (1e-3, 1.0, 3), nrhs=1)
    systems = [big, small]
    ops = _ops(systems, cuda)
    tol, otol = (1e-10, 1e-10) if prec == "fp64" else (1e-12, 1e-13)
    xs, infos, status = solve_batched(ops, [p["b"] for p in systems], tol=tol, prec=prec)
    assert status == "ok", [i["status"] for i in infos]
    t = 0
    for s, p in enumerate(systems):
        ap = O.shifted_apply(p["kind"], p["rowptr"], p["col"], p["vals"], p["n"])
        bs = np.atleast_2d(p["b"])
        for q in range(bs.shape[0]):
            ref = O.cg_m(ap, bs[q], p["sigma"], tol=otol)
            info = infos[t]
            t += 1
            assert np.all(info["true_rel_res"] <= tol), (s, q, info["true_rel_res"])
            assert np.all(_rel(xs[s][q].cpu().numpy(), ref["x"]) <= 1e-8), (s, q)
    over = W.staggered_problem((4, 4, 4, 4), 0.1, 712, 812, (1e-4, 1.0, 17), nrhs=1)
    op17 = _ops([over], cuda)
    with pytest.raises(MscError):
        solve_batched(op17, [over["b"]], tol=1e-10, prec=prec)
    for op in ops + op17:
        op.close()
