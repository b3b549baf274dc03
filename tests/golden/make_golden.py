"""Writes the stored expected values under tests/golden/ by running the CPU
oracle only (no GPU code is imported).  Usage:  python tests/golden/make_golden.py

small_uniform.json : 1000 x 1500, |Omega| = 50,000 uniform, rank-5 truth + noise
                     variance 0.01, lambda = 0.5, k0 = 8; oracle solve to relative
                     optimality residual 1e-10, with its duality-gap certificate.
netflix_quarter_lam300.json : the Netflix-shaped generator at scale 0.25 (4,442 x
                     120,047, |Omega| = 6.25e6, capped Zipf(1.2) degrees, rank-20
                     truth + noise variance 0.25 clipped to [1, 5]), lambda = 300,
                     k0 = 16; oracle solve to 1e-10 with its duality-gap certificate.

movielens100k_shape_lam15.json, toy_shape_lam36.json : the rating-shaped
                     stand-ins of synth.movielens_shape ("100k": 943 x 1,682,
                     90,570 entries, lambda 15; "toy": 3,952 x 6,040, 900,189
                     entries, lambda 36), k0 = 8; oracle solve to relative
                     optimality residual 1e-12 with its duality-gap certificate.
rke_solves.json   : the kernel-estimation QSDP oracle (oracle/rke.py) on
                     synth.rke workloads: (600 objects, 40 partners, lambda 10,
                     seed 3; k0 6, tol 1e-5, algorithm seed 1) with lmsvd_p 0
                     and 1, and the 20,000-object benchmark workload (lambda 10,
                     seed 7; k0 8, tol 1e-4, algorithm seed 1, lmsvd_p 1); final
                     F, rank, outer and subspace iterations.

    python tests/golden/make_golden.py [small_uniform] [netflix_quarter] [ml100k] [toy] [rke_600] [rke_20000]
"""
import json
import os
import sys
import time

sys.path.insert(0, os.path.abspath(os.path.join(os.path.dirname(__file__), "..", "..")))

import synth  # noqa: E402
from oracle import core, dense, rke  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def certified(p, lam, k0, seed, fname, first_at=1e-6, tol=1e-10):
    t0 = time.time()
    res = core.solve(p, core.Options(lam=lam, k0=k0, tol=tol, seed=seed, max_iter=3000),
                     callback=lambda r: print(r.t, r.F, r.residual, r.k, r.q, r.ssi_iters, flush=True))
    f, R = core.loss(p, res.W, res.H)
    gap, D, g2 = dense.duality_gap(p, R, res.F, lam)
    out = dict(problem=p.name, lam=lam, k0=k0, F=res.F, rank=res.k, residual=res.residual,
               iters=res.iters, converged=res.converged, dual_gap=gap, dual_value=D,
               grad_spectral_norm=g2, seconds=time.time() - t0,
               first_iter_at_1e6=next((r.t for r in res.history if r.residual <= first_at), None),
               note="written by tests/golden/make_golden.py from the CPU oracle")
    with open(os.path.join(HERE, fname), "w") as fh:
        json.dump(out, fh, indent=1)
    print(out)


def small_uniform():
    p = synth.small_uniform()
    certified(p, p.lam, p.k0, 11, "small_uniform.json")


def netflix_quarter():
    p = synth.netflix_shape(scale=0.25)
    certified(p, 300.0, 16, 3, "netflix_quarter_lam300.json")


def ml100k():
    p = synth.movielens_shape("100k")
    certified(p, p.lam, p.k0, 3, "movielens100k_shape_lam15.json", tol=1e-12)


def toy():
    p = synth.movielens_shape("toy")
    certified(p, p.lam, p.k0, 3, "toy_shape_lam36.json", tol=1e-12)


def _rke_case(key, n, lam, seed, k0, tol, hist, alg_seed=1):
    fname = os.path.join(HERE, "rke_solves.json")
    p = synth.rke(n, 40, lam=lam, seed=seed)
    t0 = time.time()
    r = rke.solve(p, lam, k0=k0, tol=tol, seed=alg_seed, max_iter=3000, bm_epochs=10, lmsvd_p=hist,
                  callback=lambda h: print(key, h.t, h.F, h.residual, h.k, h.ssi_iters, flush=True))
    data = json.load(open(fname)) if os.path.exists(fname) else {}
    data[key] = dict(problem=p.name, n=n, deg=40, lam=lam, seed=seed, k0=k0, tol=tol, lmsvd_p=hist,
                     alg_seed=alg_seed, bm_epochs=10, F=r.F, rank=r.k, iters=r.iters,
                     converged=r.converged, ssi_iters=sum(h.ssi_iters for h in r.history),
                     seconds=time.time() - t0,
                     note="written by tests/golden/make_golden.py from the CPU oracle")
    with open(fname, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    print(key, data[key])


def rke_600():
    for hist in (0, 1):
        _rke_case("n600_p%d" % hist, 600, 10.0, 3, 6, 1e-5, hist)


def rke_20000():
    _rke_case("n20000_p1", 20_000, 10.0, 7, 8, 1e-4, 1)


if __name__ == "__main__":
    which = sys.argv[1:] or ["small_uniform", "netflix_quarter"]
    for w in which:
        globals()[w]()
