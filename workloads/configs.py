"""The five workload recipes (sizes, masses, shifts and seeds) used by tests and bench.

c0  4^4 staggered, m=0.1, 8 shifts in [1e-4, 1], FP64           (small parity case)
c1  16^4 staggered, m=0.05, 12 shifts in [1e-5, 10]             (mixed vs FP64)
c2  32^3x64 staggered, m=0.02, 16 shifts in [1e-6, 10]          (bandwidth study)
c3  8^4 / 16^4 staggered, m=0.1, 10 shifts in [1e-4, 1]         (gradient)
c4  48 staggered systems of 4^4..12^4 + 16 Laplacians on 32^3,  (batch)
    10 shifts in [1e-4, 1], 4 right-hand sides each

Links are seeded Haar SU(3) (a stand-in for Monte Carlo gauge configurations, which
need a gauge-field ensemble this repository does not have).
"""
from __future__ import annotations

import numpy as np

from .lattice import random_su3_links, staggered_csr, lattice_volume
from .generic import gaussian_rhs, laplacian7_csr, logspace_shifts

CONFIGS = {
    "c0": dict(dims=(4, 4, 4, 4), mass=0.1, shifts=(1e-4, 1.0, 8), seed_links=1000, seed_b=2000,
               tol=1e-10),
    "c1": dict(dims=(16, 16, 16, 16), mass=0.05, shifts=(1e-5, 10.0, 12), seed_links=1001,
               seed_b=2001, tol=1e-10, reliable_every=50),
    "c2": dict(dims=(32, 32, 32, 64), mass=0.02, shifts=(1e-6, 10.0, 16), seed_links=1002,
               seed_b=2002, tol=1e-10, reliable_every=50),
    "c3": dict(dims=(8, 8, 8, 8), mass=0.1, shifts=(1e-4, 1.0, 10), seed_links=1003,
               seed_b=2003, seed_c=3003, seed_nz=4003, n_nz=32, fd_h=1e-6, tol=1e-10),
    "c3_16": dict(dims=(16, 16, 16, 16), mass=0.1, shifts=(1e-4, 1.0, 10), seed_links=1003,
                  seed_b=2003, seed_c=3003, seed_nz=4003, n_nz=32, fd_h=1e-6, tol=1e-10,
                  seed_dir=6003),
    "c3_4": dict(dims=(4, 4, 4, 4), mass=0.1, shifts=(1e-4, 1.0, 10), seed_links=1003,
                 seed_b=2003, seed_c=3003, seed_nz=4003, n_nz=32, fd_h=1e-6, tol=1e-10),
    "c4": dict(stag_dims=((4, 4, 4, 4), (6, 6, 6, 6), (8, 8, 8, 8), (12, 12, 12, 12)),
               stag_each=12, lap_dims=(32, 32, 32), lap_count=16, mass=0.1,
               shifts=(1e-4, 1.0, 10), nrhs=4, seed_links=1004, seed_b=2004, seed_mix=5004,
               tol=1e-10, reliable_every=50),
}


def staggered_problem(dims, mass, seed_links, seed_b, shifts, nrhs=None):
    """One staggered system: CSR of M, right-hand side(s) and shifts."""
    links = random_su3_links(dims, seed_links)
    rowptr, col, vals = staggered_csr(links, dims, mass)
    n = 3 * lattice_volume(dims)
    b = gaussian_rhs(n, seed_b, nrhs)
    return dict(kind="mhm", dims=tuple(dims), mass=mass, n=n, rowptr=rowptr, col=col,
                vals=vals, b=b, sigma=logspace_shifts(*shifts), links=links)


def _batch_systems(cfg):
    """The c4 batch: 48 staggered + 16 Laplacian systems in a seeded order."""
    kinds = []
    for dims in cfg["stag_dims"]:
        kinds += [("mhm", tuple(dims))] * cfg["stag_each"]
    rng = np.random.default_rng(cfg["seed_mix"])
    order = rng.permutation(len(kinds))
    kinds = [kinds[i] for i in order] + [("herm", tuple(cfg["lap_dims"]))] * cfg["lap_count"]
    sigma = logspace_shifts(*cfg["shifts"])
    systems = []
    for i, (kind, dims) in enumerate(kinds):
        seed_a = cfg["seed_links"] * 100 + i
        seed_b = cfg["seed_b"] * 100 + i
        if kind == "mhm":
            links = random_su3_links(dims, seed_a)
            rowptr, col, vals = staggered_csr(links, dims, cfg["mass"])
            n = 3 * lattice_volume(dims)
        else:
            rowptr, col, vals = laplacian7_csr(dims, seed_a)
            n = lattice_volume(dims)
        systems.append(dict(kind=kind, dims=dims, n=n, rowptr=rowptr, col=col, vals=vals,
                            b=gaussian_rhs(n, seed_b, cfg["nrhs"]), sigma=sigma))
    return systems


def make_config(name: str):
    """Materialise a named recipe: a dict with the arrays of one system (or a batch)."""
    cfg = dict(CONFIGS[name])
    if name == "c4":
        return dict(name=name, tol=cfg["tol"], systems=_batch_systems(cfg), cfg=cfg)
    prob = staggered_problem(cfg["dims"], cfg["mass"], cfg["seed_links"], cfg["seed_b"],
                             cfg["shifts"])
    prob.update(name=name, tol=cfg["tol"], cfg=cfg)
    if name.startswith("c3"):
        rng_c = np.random.default_rng(cfg["seed_c"])
        prob["c"] = rng_c.uniform(0.0, 1.0, size=cfg["shifts"][2])
        rng_nz = np.random.default_rng(cfg["seed_nz"])
        prob["fd_nz"] = np.sort(rng_nz.choice(prob["vals"].size, size=cfg["n_nz"], replace=False))
        if "seed_dir" in cfg:
            # a direction over every stored entry for a directional finite difference
            prob["fd_dir"] = gaussian_rhs(prob["vals"].size, cfg["seed_dir"])
    return prob
