"""The oracle's pins catch plausible mistakes (CPU only).

Each case plants one mistake in a copy of the oracle's CG-M source (a wrong sign, index,
power or bookkeeping step in the shifted recurrences or the driving CG) and checks that
at least one pin that holds for the real oracle fails for the copy: the dense solve, the
closed-form first step, the collinearity r_k = zeta_k r and the per-shift CG iterates.
"""
import inspect
import types

import numpy as np
import pytest

import oracle as O
import oracle.cgm as cgm_module
import workloads as W

MUTANTS = {
    "denominator sign": ("(1.0 + sh.s * a)", "(1.0 - sh.s * a)"),
    "power of the ratio in c(s)": ("(c * ratio * ratio)", "(c * ratio)"),
    "old z in the shifted direction": ("sh.d = zn * r", "sh.d = sh.z * r"),
    "current step in the z numerator": ("sh.z * sh.z_old * a_old", "sh.z * sh.z_old * a"),
    "z history not rotated": ("sh.z_old, sh.z = sh.z, zn", "sh.z_old, sh.z = zn, zn"),
    "inverted shifted step": ("(a * zn / sh.z)", "(a * sh.z / zn)"),
    "residual update sign": ("r = r - a * q", "r = r + a * q"),
    "stale direction coefficient": ("d = r + c * d", "d = r + c_old * d"),
    "coefficient from the wrong norms": ("c = rr_new / rr", "c = rr / rr_new"),
}


def _mutant(old, new):
    src = inspect.getsource(cgm_module)
    assert src.count(old) == 1, old
    mod = types.ModuleType("cgm_mutant")
    exec(compile(src.replace(old, new), "cgm_mutant", "exec"), mod.__dict__)
    return mod.cg_m


@pytest.fixture(scope="module")
def c0():
    p = W.make_config("c0")
    p["apply"] = O.shifted_apply("mhm", p["rowptr"], p["col"], p["vals"], p["n"])
    p["dense"] = O.dense_solve("mhm", p["rowptr"], p["col"], p["vals"], p["n"], p["b"], p["sigma"])
    return p


def _pins(cg_m, p):
    """Names of the pins that fail for this CG-M implementation."""
    b, ap, sigma = p["b"], p["apply"], p["sigma"]
    bn = np.linalg.norm(b)
    failed = []
    with np.errstate(all="ignore"):
        # dense solve
        try:
            res = cg_m(ap, b, sigma, tol=1e-10, max_iter=2000)
            err = np.linalg.norm(res["x"] - p["dense"], axis=1) / np.linalg.norm(p["dense"], axis=1)
            if not (res["status"] == "ok" and np.all(err <= 1e-8)):
                failed.append("dense")
        except Exception:
            failed.append("dense")
        # first step closed form and collinearity over 60 iterations
        snap, worst = {}, [0.0]

        def observe(i, r, x, zeta, order, sigma0, **_):
            if i == 1:
                snap.update(x=x.copy(), zeta=zeta.copy(), order=order, sigma0=sigma0)
            sig = sigma[order]
            for k in range(len(sig)):
                res_k = b - ap(x[k], float(sig[k]))
                worst[0] = max(worst[0], np.linalg.norm(res_k - zeta[k] * r) / bn)

        try:
            cg_m(ap, b, sigma, tol=0.0, freeze=False, observe=observe, max_iter=60)
            a0 = np.vdot(b, b).real / np.vdot(b, ap(b, snap["sigma0"])).real
            for kk, k in enumerate(snap["order"]):
                s = sigma[k] - snap["sigma0"]
                step = np.vdot(b, b).real / np.vdot(b, ap(b, float(sigma[k]))).real
                if not (abs(snap["zeta"][kk] - 1.0 / (1.0 + s * a0)) <= 1e-14
                        and np.abs(snap["x"][kk] - step * b).max() <= 1e-14 * np.abs(step * b).max()):
                    failed.append("first step")
                    break
            if not worst[0] < 1e-12:
                failed.append("collinearity")
        except Exception:
            failed.append("first step / collinearity")
        # per-shift CG iterates for 12 steps
        try:
            hist = []
            cg_m(ap, b, sigma, tol=0.0, freeze=False, max_iter=12,
                 observe=lambda i, x, order, **_: hist.append((x.copy(), order)))
            bad = False
            for k, sk in enumerate(sigma):
                ref = O.cg(ap, b, shift=float(sk), tol=0.0, max_iter=12, record=True)["history"]
                for n, (xs, order) in enumerate(hist, start=1):
                    kk = int(np.nonzero(order == k)[0][0])
                    if not np.linalg.norm(xs[kk] - ref[n]) <= 1e-9 * np.linalg.norm(ref[n]):
                        bad = True
            if bad or len(hist) != 12:
                failed.append("per-shift CG")
        except Exception:
            failed.append("per-shift CG")
    return failed


def test_real_oracle_passes_every_pin(c0):
    assert _pins(O.cg_m, c0) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_fails_a_pin(c0, name):
    old, new = MUTANTS[name]
    failed = _pins(_mutant(old, new), c0)
    assert failed, f"no pin caught the planted mistake: {name}"
