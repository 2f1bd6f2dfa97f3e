"""Benchmark: shifted-solves/s to relative residual 1e-10 on one MI355X.

A step is one complete multishift solve of the workload (all shifts to true relative
residual <= 1e-10, including the FP64 verification and, for the mixed path, the
reliable updates and per-shift refinement), with the operator and right-hand side
already resident in HBM.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload c2] [--prec mixed|fp64]

The default workload is the largest single-GPU configuration, 32^3 x 64 (c2), whose
working set is far beyond the last-level cache; 16^4 (c1), whose working set largely fits
in the 256 MB Infinity Cache, is reported beside it as cache-resident.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "shifted-solves/s & HBM GB/s to rel.residual 1e-10: mixed+batched vs FP64 plain"
PEAK_HBM_GBS = 8000.0
WORKLOAD_NAMES = {
    "c1": "16^4 staggered M^H M, m=0.05, 12 shifts in [1e-5,10], tol 1e-10",
    "c2": "32^3x64 staggered M^H M, m=0.02, 16 shifts in [1e-6,10], tol 1e-10",
    "c0": "4^4 staggered M^H M, m=0.1, 8 shifts in [1e-4,1], tol 1e-10",
}


# HBM traffic per launch comes from rocprofv3 counter runs of this same script
# (FETCH_SIZE and WRITE_SIZE, KiB per dispatch, scaled by the calibration against a copy
# kernel of known size); it is reported only while the kernel sources are unchanged since.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.json")
KERNEL_NAMES = {("mixed", "head"): "k1_fused<float, true>",
                ("mixed", "K2"): "k2_sell<float>",
                ("fp64", "head"): "k1_fused<double, true>",
                ("fp64", "K2"): "k2_sell<double>"}
# the same kernels on the matrix-free staggered operator (M and M^H from the links, one
# lattice site per lane; two rows per SU(3) link; the FP64 head forms its product by the
# recurrence t' = M r + b t in all but one launch in 64; K2 and the heads march along t
# where the lattice has enough blocks of 64 sites for it, as at 32^3x64, and not at
# 16^4): the first name that the counter summary holds for the workload
KERNEL_NAMES_MF = {("mixed", "head"): ("k1_site<float, 2, false, true>",
                                       "k1_site<float, 2, false, false>"),
                   ("mixed", "K2"): ("k2_site<float, 2, true>", "k2_site<float, 2, false>"),
                   ("fp64", "head"): ("k1_site<double, 2, true, true>",
                                      "k1_site<double, 2, true, false>"),
                   ("fp64", "K2"): ("k2_site<double, 2, true>", "k2_site<double, 2, false>")}
PHASE_NAMES = {"fp64": "FP64", "mixed": "complex64"}


def measured_traffic(workload, prec, kernel, matrix_free=False):
    """(bytes per launch, kernel name) from the committed counter summary, or (None, name)."""
    import hashlib
    names = KERNEL_NAMES_MF.get((prec, kernel)) if matrix_free else (KERNEL_NAMES.get((prec, kernel)),)
    name = names[0] if names else None
    try:
        with open(TRAFFIC_FILE) as fh:
            data = json.load(fh)
        h = hashlib.sha256()
        for rel in data["kernel_sources"]:
            with open(os.path.join(ROOT, rel), "rb") as fh:
                h.update(fh.read())
        if h.hexdigest() != data["kernel_source_sha256"]:
            return None, name
        wl = data["workloads"][workload]
        name = next((nm for nm in names if nm in wl), name)
        ent = wl[name]
        return 1024.0 * (ent["fetch_kib"] * data["fetch_scale"]
                         + ent["write_kib"] * data["write_scale"]), name
    except (OSError, KeyError, ValueError):
        return None, name


def dominant_kernel(kernels):
    """The kernel with the most GPU time per step: its average duration times its phase's
    launches (a mixed solve lists its FP64-phase and complex64-phase kernels apart)."""
    return max(kernels, key=lambda nm: kernels[nm]["ms_per_step"])


def copy_ceiling(dev, nbytes, reps=20):
    """GB/s of a device-to-device copy that reads nbytes/2 and writes nbytes/2, the mean
    of reps copies timed with events on torch's stream (after 3 untimed ones)."""
    import torch
    half = max(1, int(nbytes) // 8)
    src = torch.ones(half, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        dst.copy_(src)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    del src, dst
    return 2.0 * 4.0 * half / (ms * 1e-3) / 1e9


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# CG-M with 15 shifts on the 2-D Poisson 1000^2 matrix, ms per iteration on one Tesla T10
# (the paper's Table 1), quoted beside the same workload here as context.
PAPER_T10_MS_PER_ITER = {"fp64": 12.9839, "fp32": 8.82461}


def paper_table1_line(args, dev):
    """The paper's own benchmark workload (Table 1): the 2-D 5-point Poisson matrix on a
    1000 x 1000 grid with 15 shifts, b = 1 as in its Fig. 1 example, ms per CG-M iteration.
    The shifts are not given for Table 1; here they are 15 log-spaced in [1e-3, 1].  The
    real-valued path (msc_solve_real: double, and float with FP64 reductions for the
    paper's single-precision column) is the like-for-like comparison; the complex path on
    the same matrix (zero imaginary parts, twice the bytes) is reported beside it."""
    import torch
    import workloads as W
    from paper_1102_2143_amd import Operator

    rowptr, col, vals = W.poisson5pt_csr(1000, 1000)
    n = 1000 * 1000
    op = Operator(rowptr, col, vals, n, kind="herm", device=dev)
    sigma = W.logspace_shifts(1e-3, 1.0, 15)
    op.set_shifts(sigma)
    b = torch.ones(n, dtype=torch.complex128, device=dev)
    x = torch.empty((15, n), dtype=torch.complex128, device=dev)
    out = {"workload": "2-D Poisson 5-point 1000^2 (n = 10^6), 15 shifts log-spaced in "
                       "[1e-3, 1], b = 1, tol 1e-5 (the paper's Table 1 workload)",
           "paper_t10_ms_per_iter": PAPER_T10_MS_PER_ITER}
    # fp64: FP64 throughout; complex64: the mixed path switched at the first iteration
    # (switch_tol 1), against the paper's single-precision column
    for name, kw in (("fp64", dict(prec="fp64")), ("complex64", dict(prec="mixed", switch_tol=1.0))):
        kw = dict(tol=1e-5, max_iter=2000, verify=False, refine=False, **kw)
        op.solve(b, out=x, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        iters = 0
        for _ in range(max(1, args.steps)):
            _, info = op.solve(b, out=x, **kw)
            iters += info["iters"]
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / iters
        ref = PAPER_T10_MS_PER_ITER["fp64" if name == "fp64" else "fp32"]
        out[name] = {"ms_per_iter": round(ms, 4), "iters": info["iters"],
                     "t10_over_mi355x": round(ref / ms, 1)}
        log(f"paper workload {name}: {ms:.4f} ms per iteration ({info['iters']} iterations)")
    br = torch.ones(n, dtype=torch.float64, device=dev)
    xr = torch.empty((15, n), dtype=torch.float64, device=dev)
    for name, prec in (("real_fp64", "fp64"), ("real_single", "mixed")):
        kw = dict(tol=1e-5, max_iter=2000, verify=False, prec=prec)
        op.solve_real(br, out=xr, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        iters = 0
        for _ in range(max(1, args.steps)):
            _, info = op.solve_real(br, out=xr, **kw)
            iters += info["iters"]
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / iters
        ref = PAPER_T10_MS_PER_ITER["fp64" if prec == "fp64" else "fp32"]
        out[name] = {"ms_per_iter": round(ms, 4), "iters": info["iters"],
                     "t10_over_mi355x": round(ref / ms, 1),
                     "effective_gbs": round(info["alg_bytes"] / info["iters"] / (ms * 1e-3) / 1e9, 1)}
        log(f"paper workload {name}: {ms:.4f} ms per iteration ({info['iters']} iterations)")
    op.close()
    return out


def batched_line(args, dev):
    """The 64-system batch (4 rhs x 10 shifts each) solved in one batched call, mixed and
    FP64: shifted-solves/s and effective GB/s (algorithmic bytes / wall time)."""
    import torch
    import workloads as W
    from paper_1102_2143_amd import Operator, solve_batched

    systems = W.make_config("c4")["systems"]
    ops = []
    for p in systems:
        op = Operator(p["rowptr"], p["col"], p["vals"], p["n"], kind=p["kind"], device=dev)
        op.set_shifts(p["sigma"])
        ops.append(op)
    bs = [torch.from_numpy(np.ascontiguousarray(p["b"])).to(dev) for p in systems]
    count = sum(np.atleast_2d(p["b"]).shape[0] * p["sigma"].size for p in systems)
    out = {"workload": "c4: 48 staggered (4^4..12^4) + 16 Laplacian 32^3 systems, 4 rhs, "
                       "10 shifts each, tol 1e-10", "shifted_solves": int(count)}
    for prec in ("mixed", "fp64"):
        for _ in range(args.warmup):
            solve_batched(ops, bs, tol=1e-10, prec=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ok = True
        for _ in range(args.steps):
            _, infos, status = solve_batched(ops, bs, tol=1e-10, prec=prec)
            ok = ok and status == "ok" and all(i["true_rel_res"].max() <= 1e-10 for i in infos)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / args.steps
        ab = sum(i["alg_bytes"] for i in infos)
        out[prec] = {"ms_per_step": round(1e3 * wall, 3), "value": round(count / wall, 1),
                     "effective_gbs": round(ab / wall / 1e9, 1), "converged": bool(ok),
                     "max_iters": max(i["iters"] for i in infos)}
        log(f"batched {prec}: {1e3 * wall:.1f} ms per batch, ok={ok}")
    out["mixed_speedup"] = round(out["fp64"]["ms_per_step"] / out["mixed"]["ms_per_step"], 3)
    for op in ops:
        op.close()
    return out


def cpu_model():
    """The host CPU's model name from /proc/cpuinfo (else what platform reports)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline(prob, sample_iters, full_iters):
    """Time the FP64 oracle on a bounded sample of the same solve (single thread): the
    first `sample_iters` iterations of its CG-M on the same operator, shifts and b, with
    its own set-up (CSR and M^H) and the final residual check left out of the timing; the
    solve's cost is the measured time per iteration times the FP64 iteration count."""
    import oracle as O
    from threadpoolctl import threadpool_limits

    ap = O.shifted_apply("mhm", prob["rowptr"], prob["col"], prob["vals"], prob["n"])
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        res = O.cg_m(ap, prob["b"], prob["sigma"], tol=prob["tol"], max_iter=sample_iters,
                     verify=False)
        dt = time.perf_counter() - t0
    done = max(1, res["iters"])
    per_iter = dt / done
    est = per_iter * full_iters
    ns = prob["sigma"].size
    return {"value": ns / est, "unit": "shifted-solves/s", "cores": 1, "kind": "oracle",
            "sample": (f"oracle CG-M (numpy/scipy FP64, 1 thread) on the same operator, "
                       f"shifts and b: the first {done} of the {full_iters} iterations of "
                       f"the FP64 solve, {dt:.1f} s ({1e3 * per_iter:.0f} ms per iteration, "
                       f"set-up and final residual check excluded), scaled to the full "
                       f"iteration count: {est:.0f} s per solve"),
            "s_per_iter": per_iter, "est_s_per_solve": est,
            "host_cpus": os.cpu_count(), "cpu_model": cpu_model()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOAD_NAMES))
    ap.add_argument("--prec", default="both", choices=["fp64", "mixed", "both"],
                    help="both: time the FP64 plain solve and the mixed solve (the headline)")
    ap.add_argument("--timing", type=int, default=128,
                    help="time the kernels of a run of consecutive iterations (one folding "
                         "cycle of the shift update) out of every k with dispatch events")
    ap.add_argument("--cpu-sample-iters", type=int, default=0,
                    help="oracle iterations timed for cpu_baseline (0: about 10-30 s of one "
                         "core: 8 at 32^3x64, 420 at 16^4, all at 4^4)")
    ap.add_argument("--fp64-steps", type=int, default=5,
                    help="timed steps of the FP64 plain comparison line (after one warm-up)")
    ap.add_argument("--no-matrix-free", action="store_true",
                    help="skip the matrix-free staggered operator's lines (links instead of "
                         "a stored matrix in the iteration)")
    ap.add_argument("--headline-op", default="matrix_free", choices=["stored", "matrix_free"],
                    help="which operator the headline value is quoted on")
    ap.add_argument("--no-c1", action="store_true",
                    help="skip the cache-resident 16^4 line reported beside the 32^3x64 one")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 64-system batched solve reported beside the main line")
    ap.add_argument("--no-paper-workload", action="store_true",
                    help="skip the paper's Table 1 workload (2-D Poisson) reported beside it")
    ap.add_argument("--no-copy-ceiling", action="store_true",
                    help="skip the copy-kernel ceiling beside the roofline figures")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="copy this many MiB once before timing (a kernel of known traffic "
                         "that calibrates FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(the solve would shard by lattice rows with a halo exchange)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    from paper_1102_2143_amd import Operator

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    prob = W.make_config(args.workload)
    log(f"generated {args.workload}: n={prob['n']} nnz={prob['vals'].size} "
        f"ns={prob['sigma'].size} in {time.perf_counter() - t0:.1f}s")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    op = Operator(prob["rowptr"], prob["col"], prob["vals"], prob["n"], kind="mhm", device=dev)
    op.set_shifts(prob["sigma"])
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    b = torch.from_numpy(prob["b"]).to(dev)
    x = torch.empty((prob["sigma"].size, prob["n"]), dtype=torch.complex128, device=dev)
    if args.copy_probe_mb > 0:
        src = torch.ones(args.copy_probe_mb << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe_mb} MiB read + {args.copy_probe_mb} MiB written")
        del src, dst

    def run_path(prec, steps, warmup, prob=prob, op=op, b=b, x=x, fmt="auto"):
        kw = dict(tol=prob["tol"], prec=prec, timing=args.timing, format=fmt)
        for i in range(warmup):
            _, info = op.solve(b, out=x, **kw)
            log(f"{prec} warmup {i}: {info['status']} iters={info['iters']} {info['seconds']:.4f}s")
        torch.cuda.synchronize()
        infos = []
        t0 = time.perf_counter()
        for i in range(steps):
            _, info = op.solve(b, out=x, **kw)
            infos.append(info)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        for i, info in enumerate(infos):
            log(f"{prec} step {i}: {info['status']} iters={info['iters']} refine={info['refine_iters']} "
                f"refined={info['n_refined']} max true res={info['true_rel_res'].max():.3e} "
                f"{info['seconds']:.4f}s")
        ok = all(inf["status"] == "ok" and inf["true_rel_res"].max() <= prob["tol"] for inf in infos)
        ns = prob["sigma"].size
        n, nnz = prob["n"], prob["vals"].size
        iters = infos[-1]["iters"]
        alg_bytes = float(np.mean([inf["alg_bytes"] for inf in infos]))
        # a mixed solve reports its FP64 phase apart from its complex64 phase; each phase
        # launches one of each iteration kernel per iteration
        it64 = float(np.mean([inf["iters_fp64"] for inf in infos]))
        itall = float(np.mean([inf["iters"] for inf in infos]))
        if prec == "mixed":
            phases = [("fp64", "fp64_kernel", it64), ("mixed", "kernel", itall - it64)]
        else:
            phases = [("fp64", "kernel", itall)]
        kernels = {}
        for phase, key, launches in phases:
            samples = sum(inf[key + "_samples"] for inf in infos)
            if samples == 0:
                continue
            kms = np.sum([inf[key + "_ms"] for inf in infos], axis=0)
            kby = np.sum([inf[key + "_bytes"] for inf in infos], axis=0)
            # slot 2 (a separate update kernel) is empty when the update is fused into the head
            names = ["head", "K2"] if kms[2] == 0 else ["K1", "K2", "K3"]
            for k, nm in enumerate(names):
                # algorithmic bytes of the sampled launches (the library counts the shifts
                # active at each sampled iteration) over their measured durations; the
                # kernel's time per step is its average duration times the phase's launches
                avg_us = 1e3 * kms[k] / samples
                kernels[f"{PHASE_NAMES[phase]} {nm}"] = {
                    "phase": phase, "kernel": nm, "avg_us": round(avg_us, 2),
                    "alg_bytes": round(kby[k] / samples),
                    "gbs": round(kby[k] / (kms[k] * 1e-3) / 1e9, 1),
                    "launches_per_step": round(launches, 1),
                    "ms_per_step": round(1e-3 * avg_us * launches, 3)}
        return dict(prec=prec, wall=wall, ok=ok, iters=iters, infos=infos, fmt=fmt,
                    value=ns * steps / wall, ms_per_step=1e3 * wall / steps, steps=steps,
                    eff_gbs=alg_bytes / (wall / steps) / 1e9, kernels=kernels,
                    refine_iters=infos[-1]["refine_iters"], n_refined=infos[-1]["n_refined"],
                    max_res=float(max(inf["true_rel_res"].max() for inf in infos)))

    # the headline path takes --steps / --warmup; the FP64 plain comparison beside it takes
    # --fp64-steps after one warm-up
    def run_op(op, fmt, headline):
        """The mixed and FP64 paths on one operator; the headline one takes --steps /
        --warmup, the other --fp64-steps (FP64) or up to 10 steps after one warm-up."""
        out = {}
        if args.prec in ("mixed", "both"):
            st = args.steps if headline else min(args.steps, 10)
            out["mixed"] = run_path("mixed", st, args.warmup if headline else 1, op=op, fmt=fmt)
        if args.prec in ("fp64", "both"):
            fp64_only = args.prec == "fp64"
            out["fp64"] = run_path("fp64", args.steps if fp64_only and headline else args.fp64_steps,
                                   args.warmup if fp64_only and headline else 1, op=op, fmt=fmt)
        return out

    # the stored matrix (CSR handed to msc_op_create_csr; the iteration reads its sliced
    # ELLPACK copies) and, for the staggered workloads, the matrix-free operator built
    # from the links (msc_op_create_staggered; the iteration reads the links)
    want_mf = not args.no_matrix_free and "links" in prob
    headline_mf = args.headline_op == "matrix_free" and want_mf
    res_stored = run_op(op, "auto", not headline_mf)
    op.close()
    del op
    res_mf, mf_setup_s = None, None
    if want_mf:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        op_mf = Operator.staggered(prob["links"], prob["dims"], prob["mass"], device=dev)
        op_mf.set_shifts(prob["sigma"])
        torch.cuda.synchronize()
        mf_setup_s = time.perf_counter() - t0
        res_mf = run_op(op_mf, "stencil", headline_mf)
        op_mf.close()
        del op_mf
    res = res_mf if headline_mf else res_stored
    paths = list(res)
    main_path = res["mixed"] if "mixed" in res else res[paths[0]]
    kernels = main_path["kernels"]
    roofline = None
    if kernels:
        dom = dominant_kernel(kernels)
        ach = kernels[dom]["gbs"]
        traffic, kname = measured_traffic(args.workload, kernels[dom]["phase"],
                                          kernels[dom]["kernel"], matrix_free=headline_mf)
        roofline = {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "frac": round(ach / PEAK_HBM_GBS, 4),
                    "traffic": None if traffic is None else round(traffic),
                    "kernel": dom, "kernel_name": kname,
                    "alg_bytes": kernels[dom]["alg_bytes"],
                    "kernel_avg_us": kernels[dom]["avg_us"],
                    "kernel_ms_per_step": kernels[dom]["ms_per_step"]}
        if not args.no_copy_ceiling:
            same = copy_ceiling(dev, kernels[dom]["alg_bytes"])
            big = copy_ceiling(dev, 2 << 30)
            roofline["copy_ceiling"] = {
                "same_bytes_gbs": round(same, 1), "2GiB_gbs": round(big, 1),
                "frac_of_same_bytes": round(ach / same, 4),
                "note": "device-to-device copy moving the kernel's algorithmic bytes (half "
                        "read, half written; a working set of that size stays partly in "
                        "the last-level cache, as the kernel's does), and 2 GiB beyond it"}
    ns = prob["sigma"].size
    n, nnz = prob["n"], prob["vals"].size
    iters = main_path["iters"]
    c1_line = None
    if args.workload == "c2" and not args.no_c1:
        # 16^4: the working set (about 0.2 GB) largely fits the 256 MB last-level cache, so
        # its rates are cache-resident rates, not HBM bandwidth
        p1 = W.make_config("c1")
        op1 = Operator(p1["rowptr"], p1["col"], p1["vals"], p1["n"], kind="mhm", device=dev)
        op1.set_shifts(p1["sigma"])
        b1 = torch.from_numpy(p1["b"]).to(dev)
        x1 = torch.empty((p1["sigma"].size, p1["n"]), dtype=torch.complex128, device=dev)
        st1 = min(args.steps, 10)
        r1 = {pp: run_path(pp, st1, 1, prob=p1, op=op1, b=b1, x=x1) for pp in ("mixed", "fp64")}
        c1_line = {"workload": f"c1: {WORKLOAD_NAMES['c1']}",
                   "note": "cache-resident: the working set largely fits the 256 MB "
                           "last-level cache; effective GB/s here is not HBM bandwidth",
                   "steps": st1}
        for pp, rr in r1.items():
            c1_line[pp] = {"value": round(rr["value"], 3), "ms_per_step": round(rr["ms_per_step"], 3),
                           "iters": rr["iters"], "converged": rr["ok"],
                           "max_true_rel_res": rr["max_res"],
                           "effective_gbs": round(rr["eff_gbs"], 1)}
        c1_line["mixed_speedup"] = round(r1["mixed"]["value"] / r1["fp64"]["value"], 3)
        op1.close()
        del op1, b1, x1
    cpu = None
    if not args.no_cpu_baseline:
        sample = args.cpu_sample_iters or {"c2": 8, "c1": 420}.get(args.workload, 100000)
        log(f"cpu baseline: oracle for {sample} iterations")
        ref_iters = res["fp64"]["iters"] if "fp64" in res else iters
        cpu = cpu_baseline(prob, sample, ref_iters)
    fp64 = res.get("fp64")

    def summary(rr):
        """The mixed and FP64 lines of one operator form, beside the headline."""
        if rr is None:
            return None
        out = {}
        for pp, r in rr.items():
            out[pp] = {"value": round(r["value"], 3), "ms_per_step": round(r["ms_per_step"], 3),
                       "steps": r["steps"], "iters": r["iters"], "converged": r["ok"],
                       "max_true_rel_res": r["max_res"], "effective_gbs": round(r["eff_gbs"], 1),
                       "kernels": r["kernels"]}
        if "mixed" in rr and "fp64" in rr:
            out["mixed_speedup"] = round(rr["mixed"]["value"] / rr["fp64"]["value"], 3)
        return out

    other = res_stored if headline_mf else res_mf
    other_line = summary(other)
    if other_line is not None:
        other_line["operator"] = ("stored matrix: CSR to msc_op_create_csr, iteration on its "
                                  "sliced ELLPACK copies" if headline_mf else
                                  "matrix-free: links to msc_op_create_staggered, iteration "
                                  "applies M and M^H from the links")
        other_line["setup_s"] = round(setup_s if headline_mf else mf_setup_s, 3)
        other_line["vs_headline"] = round(other["mixed"]["value"] / main_path["value"], 3) \
            if "mixed" in other and main_path["prec"] == "mixed" else None
    line = {
        "metric": METRIC,
        "value": round(main_path["value"], 3),
        "unit": "shifted-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_path["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_path["prec"] == "fp64" else "f32+f64",
        "data": "synthetic (seeded Haar SU(3) links, complex Gaussian b)",
        "config": {"workload": f"{args.workload}: {WORKLOAD_NAMES[args.workload]}", "n": n,
                   "nnz_M": nnz, "ns": ns, "prec": main_path["prec"], "iters": iters,
                   "operator": "matrix_free" if headline_mf else "stored",
                   "refine_iters": main_path["refine_iters"], "n_refined": main_path["n_refined"],
                   "parallelism": "single GPU"},
        "converged": main_path["ok"],
        "max_true_rel_res": main_path["max_res"],
        "effective_gbs": round(main_path["eff_gbs"], 1),
        "iters_per_s": round(iters * args.steps / main_path["wall"], 1),
        "setup_s": round(mf_setup_s if headline_mf else setup_s, 3),
        "kernels": kernels,
        "fp64_plain": None if fp64 is None or fp64 is main_path else {
            "value": round(fp64["value"], 3), "ms_per_step": round(fp64["ms_per_step"], 3),
            "steps": fp64["steps"],
            "iters": fp64["iters"], "converged": fp64["ok"], "max_true_rel_res": fp64["max_res"],
            "effective_gbs": round(fp64["eff_gbs"], 1), "kernels": fp64["kernels"],
            "mixed_speedup": round(main_path["value"] / fp64["value"], 3)},
        "roofline": roofline,
        ("stored_matrix" if headline_mf else "matrix_free"): other_line,
        "cpu_baseline": cpu,
        "c1_cache_resident": c1_line,
        "batched": None if args.no_batch else batched_line(args, dev),
        "paper_table1": None if args.no_paper_workload else paper_table1_line(args, dev),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
