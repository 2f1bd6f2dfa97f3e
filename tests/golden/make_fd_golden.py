"""Write the finite-difference gradient fixture of the 8^4 gradient workload.

Calls only the oracle (test infrastructure): central differences with h = 1e-6 of the
second-order functional L~ = sum_k c_k Re(b^H x_k + x_k^H r_k) (x_k from the FP64 CG-M
oracle at tol 1e-14), for the real and imaginary part of 32 seeded stored entries of M;
with the argument ``directional``, the 16^4 fixture: one central difference along a seeded
direction over every stored entry; with ``entries16`` the 16^4 fixture of 32 seeded stored
entries, real and imaginary part each (128 oracle solves, spread over worker processes);
with ``loss`` the loss L~ at the unperturbed entries is added to the per-entry fixtures
(the scale of the central differences' rounding error, u |L~| / h).
The loss is the rational-approximation form sum_k c_k Re(b^H x_k) of the shifted family
(Section 2 of the paper).
Run:  python tests/golden/make_fd_golden.py [directional | entries16 [jobs] | loss]
"""
import concurrent.futures
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402


def base_loss(name):
    """L~ at the unperturbed entries (one FP64 CG-M oracle solve at tol 1e-14)."""
    p = W.make_config(name)
    ap = O.shifted_apply("mhm", p["rowptr"], p["col"], p["vals"], p["n"])
    sol = O.cg_m(ap, p["b"], p["sigma"], tol=1e-14, max_iter=100000)
    return O.second_order_loss("mhm", p["rowptr"], p["col"], p["vals"], p["n"], p["b"],
                               p["sigma"], p["c"], sol["x"])


def main_loss():
    for name, out in (("c3", "fd_c3_8x4.json"), ("c3_16", "fd_c3_16x4.json")):
        path = os.path.join(HERE, out)
        rec = json.load(open(path))
        rec["loss"] = float(base_loss(name))
        with open(path, "w") as f:
            json.dump(rec, f, indent=1)
        print(f"{out}: loss {rec['loss']:.6e}")


def main(name="c3", out="fd_c3_8x4.json"):
    p = W.make_config(name)
    cfg = p["cfg"]
    t0 = time.time()
    fd = O.fd_gradient("mhm", p["rowptr"], p["col"], p["vals"], p["n"], p["b"], p["sigma"], p["c"],
                       p["fd_nz"], h=cfg["fd_h"], tol=1e-14)
    rec = dict(config=name, dims=list(cfg["dims"]), mass=cfg["mass"], shifts=list(cfg["shifts"]),
               seeds=dict(links=cfg["seed_links"], b=cfg["seed_b"], c=cfg["seed_c"], nz=cfg["seed_nz"]),
               h=cfg["fd_h"], solve_tol=1e-14, nz=[int(e) for e in p["fd_nz"]],
               grad_re=[float(v.real) for v in fd], grad_im=[float(v.imag) for v in fd],
               loss=float(base_loss(name)), seconds=round(time.time() - t0, 1),
               source="oracle.fd_gradient (central differences of the second-order functional)")
    with open(os.path.join(HERE, out), "w") as f:
        json.dump(rec, f, indent=1)
    print(f"wrote {out} in {time.time() - t0:.0f}s")


def main_directional(name="c3_16", out="fd_c3_16x4_dir.json"):
    """The 16^4 gradient workload: one central difference of L~ along a seeded complex
    Gaussian direction over every stored entry of M (two oracle solves)."""
    p = W.make_config(name)
    cfg = p["cfg"]
    t0 = time.time()
    d = O.fd_directional("mhm", p["rowptr"], p["col"], p["vals"], p["n"], p["b"], p["sigma"],
                         p["c"], p["fd_dir"], h=cfg["fd_h"], tol=1e-14)
    rec = dict(config=name, dims=list(cfg["dims"]), mass=cfg["mass"], shifts=list(cfg["shifts"]),
               seeds=dict(links=cfg["seed_links"], b=cfg["seed_b"], c=cfg["seed_c"],
                          direction=cfg["seed_dir"]),
               h=cfg["fd_h"], solve_tol=1e-14, directional_derivative=float(d),
               seconds=round(time.time() - t0, 1),
               source="oracle.fd_directional (central difference of the second-order "
                      "functional along workloads.gaussian_rhs(nnz, seed_dir))")
    with open(os.path.join(HERE, out), "w") as f:
        json.dump(rec, f, indent=1)
    print(f"wrote {out} in {time.time() - t0:.0f}s")


def _one_entry(args):
    name, e = args
    p = W.make_config(name)
    cfg = p["cfg"]
    g = O.fd_gradient("mhm", p["rowptr"], p["col"], p["vals"], p["n"], p["b"],
                      p["sigma"], p["c"], [e], h=cfg["fd_h"], tol=1e-14)
    return e, complex(g[0])


def main_entries16(name="c3_16", out="fd_c3_16x4.json", jobs=8):
    """The 16^4 gradient workload, per entry: central differences for the real and the
    imaginary part of each of the 32 seeded stored entries (the 8^4 recipe at 16^4)."""
    p = W.make_config(name)
    cfg = p["cfg"]
    nz = [int(e) for e in p["fd_nz"]]
    t0 = time.time()
    res = {}
    with concurrent.futures.ProcessPoolExecutor(max_workers=jobs) as ex:
        for e, g in ex.map(_one_entry, [(name, e) for e in nz]):
            res[e] = g
            print(f"entry {e}: {g.real:.12e} {g.imag:.12e}  ({time.time() - t0:.0f}s)", flush=True)
    rec = dict(config=name, dims=list(cfg["dims"]), mass=cfg["mass"], shifts=list(cfg["shifts"]),
               seeds=dict(links=cfg["seed_links"], b=cfg["seed_b"], c=cfg["seed_c"], nz=cfg["seed_nz"]),
               h=cfg["fd_h"], solve_tol=1e-14, nz=nz,
               grad_re=[float(res[e].real) for e in nz], grad_im=[float(res[e].imag) for e in nz],
               loss=float(base_loss(name)), seconds=round(time.time() - t0, 1),
               source="oracle.fd_gradient (central differences of the second-order functional)")
    with open(os.path.join(HERE, out), "w") as f:
        json.dump(rec, f, indent=1)
    print(f"wrote {out} in {time.time() - t0:.0f}s")


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "directional":
        main_directional()
    elif len(sys.argv) > 1 and sys.argv[1] == "loss":
        main_loss()
    elif len(sys.argv) > 1 and sys.argv[1] == "entries16":
        main_entries16(jobs=int(sys.argv[2]) if len(sys.argv) > 2 else 8)
    else:
        main()
