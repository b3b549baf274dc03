"""GPU parity of the kernel-estimation QSDP path (bmg_rke_*) against
oracle/rke.py on the same seeded inputs (FP64).  Tolerances: pair residuals
4 k u (|w_i|^2 + |w_j|^2 + d^2) elementwise; solves: objective within 1e-8
relative, the same rank."""
import json
import math
import os

import numpy as np
import pytest
import torch

import paper_2204_14067_amd as bmg
import synth
from oracle import rke

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
U = 2.0 ** -53


def to_dev(p, k_cap=32, precision="fp64", lmsvd_p=0):
    return bmg.Problem.from_host(p.row_ptr, p.col, p.val, p.m, p.n, k_cap=k_cap, precision=precision,
                                 device=DEV, lmsvd_p=lmsvd_p)


@pytest.mark.parametrize("n,deg,k", [(30, 8, 1), (200, 20, 5), (3000, 5000, 17)])
def test_rke_residual_parity(n, deg, k):
    """(3000, 5000): rows longer than one piece (split and summed in order)."""
    p = synth.rke(n, deg, seed=n)
    print("rke residual", n, p.nnz, k, flush=True)
    dp = to_dev(p, k_cap=32)
    W = np.zeros((n, 32))
    W[:, :k] = np.random.default_rng(k).standard_normal((n, k))
    r, dg, s2 = dp.bmg_rke_residual(torch.as_tensor(W, device=DEV), k)
    ro = rke.pair_residual(p, W[:, :k])
    rows = p.rows()
    nrm = np.sum(W[:, :k] ** 2, axis=1)
    bound = 4 * k * U * (nrm[rows] + nrm[p.col] + np.abs(p.val)) * 4
    assert np.all(np.abs(r.cpu().numpy() - ro) <= bound + 1e-300)
    dgo = np.bincount(rows, weights=ro, minlength=n)
    assert np.allclose(dg.cpu().numpy(), dgo, rtol=1e-12, atol=1e-9)
    assert math.isclose(s2, float(ro @ ro), rel_tol=1e-12)


@pytest.mark.parametrize("hist", [0, 1])
@pytest.mark.parametrize("n,deg,lam", [(50, 30, 2.0), (100, 30, 1.5)])
def test_rke_solve_parity(n, deg, lam, hist):
    """Plain subspace iteration (lmsvd_p 0) and Algorithm 2 with history 1,
    both with the rank safeguard column of eq. rt."""
    p = synth.rke(n, deg, lam=lam, seed=3)
    orc = rke.solve(p, lam, k0=6, tol=1e-8, seed=1, max_iter=1000, lmsvd_p=hist)
    dp = to_dev(p, k_cap=64, lmsvd_p=hist)
    W, k, r = dp.bmg_rke_solve(lam=lam, k_init=6, tol=1e-8, seed=1, max_iter=1000, bm_epochs=10,
                               lmsvd_p=hist)
    print("rke solve", n, hist, r["iters"], orc.iters, r["F"], orc.F, k, orc.k, r["ssi_iters"],
          sum(h.ssi_iters for h in orc.history), flush=True)
    assert r["status"] == 0 and orc.converged
    assert math.isclose(r["F"], orc.F, rel_tol=1e-8)
    assert k == orc.k
    Wg = W.cpu().numpy()[:, :k]
    assert np.allclose(Wg.sum(axis=0), 0.0, atol=1e-8 * max(1.0, np.abs(Wg).max()))
    assert math.isclose(rke.objective(p, Wg, lam), r["F"], rel_tol=1e-10)


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "rke_solves.json")


@pytest.mark.parametrize("key", ["n600_p0", "n600_p1"])
def test_rke_solve_against_stored_oracle_solves(key):
    """A workload of the benchmark's shape (noisy distances, the rank growing
    over the solve), too slow for the oracle at test time: its solves are
    stored by tests/golden/make_golden.py.  The same objective to 1e-8 and the
    rank to within one (see below).  The iteration counts are printed, not compared: the newest Ritz
    vector lies in a cluster of eigenvalues and is fixed by rounding, so the two
    trajectories part after a few steps and meet again at the optimum (at tol
    1e-5 both are within 1e-9 of it)."""
    stored = json.load(open(GOLDEN)) if os.path.exists(GOLDEN) else {}
    if key not in stored:
        pytest.skip("no stored oracle solve for " + key)
    g = stored[key]
    p = synth.rke(g["n"], g["deg"], lam=g["lam"], seed=g["seed"])
    dp = to_dev(p, k_cap=160, lmsvd_p=g["lmsvd_p"])
    W, k, r = dp.bmg_rke_solve(lam=g["lam"], k_init=g["k0"], tol=g["tol"], seed=g["alg_seed"],
                               max_iter=3000, bm_epochs=g["bm_epochs"], lmsvd_p=g["lmsvd_p"])
    print("rke stored", key, r["iters"], g["iters"], r["F"], g["F"], k, g["rank"], r["ssi_iters"],
          g["ssi_iters"], "ssi per PG step %.2f" % (r["ssi_iters"] / (r["iters"] + 1)), flush=True)
    assert r["status"] == 0 and g["converged"]
    assert math.isclose(r["F"], g["F"], rel_tol=1e-8)
    # the optimum's 25th eigenvalue is close to 0 here: which side of the cut
    # it ends on at tol 1e-5 depends on the trajectory (both sides reach F to
    # 1e-8), so the rank is compared to within one
    assert abs(k - g["rank"]) <= 1


def test_rke_benchmark_workload_solve_is_an_oracle_optimality_point():
    """The benchmark workload itself (20,000 objects, about 40 partners each,
    lambda 10, lmsvd_p 1, tol 1e-4).  Its trajectory is fixed by rounding (see
    above), so the check is on the point returned, with the oracle's own
    functions: the objective to 1e-10, and the oracle's stop residual of one
    exact PG step from it within 3 x tol.  The subspace iterations average at
    most 20 per PG step; the stored oracle solve of the same workload (its own
    trajectory) ends within 1e-3 of the same objective."""
    p = synth.rke(20_000, 40, lam=10.0, seed=7)
    lam, tol = 10.0, 1e-4
    dp = to_dev(p, k_cap=160, lmsvd_p=1)
    W, k, r = dp.bmg_rke_solve(lam=lam, k_init=8, tol=tol, seed=1, max_iter=3000, bm_epochs=10, lmsvd_p=1)
    per_step = r["ssi_iters"] / (r["iters"] + 1)
    assert r["status"] == 0
    Wh = W.cpu().numpy()[:, :k]
    Fo = rke.objective(p, Wh, lam)
    alpha = 1.99 / rke.lipschitz_bound(p)
    ro = rke.pair_residual(p, Wh)
    U0 = np.column_stack([Wh, np.random.default_rng(5).standard_normal(p.n)])
    ep = rke.eig_prox(p, Wh, ro, alpha, lam, U0, 1e-10, max_iter=400, p=1)
    res_o = rke.stop_residual(p, Wh, ep.W, ro, alpha, lam)
    stored = json.load(open(GOLDEN)).get("n20000_p1", {}) if os.path.exists(GOLDEN) else {}
    print("rke 20000: iters", r["iters"], "rank", k, "F", r["F"], "oracle F(W)", Fo, "oracle residual",
          res_o, "ssi per PG step %.2f" % per_step, "stored oracle solve", stored.get("F"),
          stored.get("rank"), stored.get("iters"), flush=True)
    assert math.isclose(Fo, r["F"], rel_tol=1e-10)
    assert res_o <= 3 * tol
    assert per_step <= 20
    if stored:
        assert abs(r["F"] - stored["F"]) <= 1e-3 * stored["F"]


def test_rke_rejects_unsymmetric_and_reduced_precision():
    p = synth.tiny(20, 20, 100, seed=3)            # a square but unsymmetric Omega
    dp = to_dev(p, k_cap=8)
    with pytest.raises(bmg.BmgError, match="BMG_EINVAL"):
        dp.bmg_rke_solve(lam=1.0)
    q = synth.rke(30, 8, seed=4)
    with pytest.raises(bmg.BmgError, match="BMG_EINVAL"):
        to_dev(q, k_cap=8, precision="fp32").bmg_rke_solve(lam=1.0)
    with pytest.raises(bmg.BmgError, match="BMG_EINVAL"):
        to_dev(q, k_cap=8).bmg_rke_solve(lam=-1.0)
    with pytest.raises(bmg.BmgError, match="BMG_EINVAL"):
        to_dev(q, k_cap=8, lmsvd_p=2).bmg_rke_solve(lam=1.0, lmsvd_p=2)
    # history blocks the workspace was not sized for
    with pytest.raises(bmg.BmgError, match="BMG_ENOMEM"):
        to_dev(q, k_cap=8).bmg_rke_solve(lam=1.0, lmsvd_p=1)
