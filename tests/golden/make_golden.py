"""Writes the stored expected values under tests/golden/ by running the CPU
oracle only (no GPU code is imported).  Usage:  python tests/golden/make_golden.py

small_uniform.json : 1000 x 1500, |Omega| = 50,000 uniform, rank-5 truth + noise
                     variance 0.01, lambda = 0.5, k0 = 8; oracle solve to relative
                     optimality residual 1e-10, with its duality-gap certificate.
"""
import json
import os
import sys
import time

sys.path.insert(0, os.path.abspath(os.path.join(os.path.dirname(__file__), "..", "..")))

import synth  # noqa: E402
from oracle import core, dense  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def small_uniform():
    p = synth.small_uniform()
    t0 = time.time()
    res = core.solve(p, core.Options(lam=p.lam, k0=p.k0, tol=1e-10, seed=11, max_iter=3000),
                     callback=lambda r: print(r.t, r.F, r.residual, r.k, r.q, r.ssi_iters, flush=True))
    f, R = core.loss(p, res.W, res.H)
    gap, D, g2 = dense.duality_gap(p, R, res.F, p.lam)
    out = dict(problem=p.name, lam=p.lam, k0=p.k0, F=res.F, rank=res.k, residual=res.residual,
               iters=res.iters, converged=res.converged, dual_gap=gap, dual_value=D,
               grad_spectral_norm=g2, seconds=time.time() - t0,
               first_iter_at_1e6=next((r.t for r in res.history if r.residual <= 1e-6), None),
               note="written by tests/golden/make_golden.py from the CPU oracle")
    with open(os.path.join(HERE, "small_uniform.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(out)


if __name__ == "__main__":
    small_uniform()
