"""Writes the stored expected values under tests/golden/ by running the CPU
oracle only (no GPU code is imported).  Usage:  python tests/golden/make_golden.py

small_uniform.json : 1000 x 1500, |Omega| = 50,000 uniform, rank-5 truth + noise
                     variance 0.01, lambda = 0.5, k0 = 8; oracle solve to relative
                     optimality residual 1e-10, with its duality-gap certificate.
netflix_quarter_lam300.json : the Netflix-shaped generator at scale 0.25 (4,442 x
                     120,047, |Omega| = 6.25e6, capped Zipf(1.2) degrees, rank-20
                     truth + noise variance 0.25 clipped to [1, 5]), lambda = 300,
                     k0 = 16; oracle solve to 1e-10 with its duality-gap certificate.

    python tests/golden/make_golden.py [small_uniform] [netflix_quarter]
"""
import json
import os
import sys
import time

sys.path.insert(0, os.path.abspath(os.path.join(os.path.dirname(__file__), "..", "..")))

import synth  # noqa: E402
from oracle import core, dense  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def certified(p, lam, k0, seed, fname, first_at=1e-6):
    t0 = time.time()
    res = core.solve(p, core.Options(lam=lam, k0=k0, tol=1e-10, seed=seed, max_iter=3000),
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


if __name__ == "__main__":
    which = sys.argv[1:] or ["small_uniform", "netflix_quarter"]
    for w in which:
        globals()[w]()
