"""GPU parity: every entry point of libbmg.so against the CPU oracle on the same
seeded inputs (FP64 unless stated).

Tolerances:
* sampled residual: |R_gpu - R_orc| <= 4 k u (|W| |H|^T + |A|)_ij elementwise,
  u = 2^-53 (the two sides add the k products in different orders);
* sparse products: |C_gpu - C_orc| <= 4 d u (|S| |B|)  with d the row length;
* iterative results (BM epochs, prox, solve): relative objective error
  <= 1e-8 in FP64 and <= 1e-5 in FP32, the bars the method is held to.
"""
import json
import math
import os

import numpy as np
import pytest
import torch

import paper_2204_14067_amd as bmg
import synth
from oracle import core, dense

pytestmark = pytest.mark.gpu
U = 2.0 ** -53
DEV = "cuda:0"


def to_dev(p, k_cap=32, precision="fp64", **reserve):
    """reserve: lmsvd_p / sparsa, the variants the workspace is sized for."""
    return bmg.Problem.from_host(p.row_ptr, p.col, p.val, p.m, p.n, k_cap=k_cap,
                                 precision=precision, device=DEV, **reserve)


def factors(p, k, ld, seed):
    rng = np.random.default_rng(seed)
    W = np.zeros((p.m, ld)); H = np.zeros((p.n, ld))
    W[:, :k] = rng.standard_normal((p.m, k))
    H[:, :k] = rng.standard_normal((p.n, k))
    return W, H


def t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def long_rows_problem():
    row_ptr, col = synth.uniform_pattern(12, 9000, 36_000, seed=21)   # rows of ~3000 > one piece
    val, _, _ = synth.values(12, 9000, row_ptr, col, 3, 0.5, 0.01, seed=22)
    return synth.Problem("long_rows", 12, 9000, row_ptr, col, val, 0.3, 4)


CASES = {
    "tiny": lambda: synth.tiny(7, 11, 30),
    "single_entry": lambda: synth.tiny(3, 4, 1),
    "empty_rows": lambda: synth.tiny(80, 50, 40, seed=4),
    "tall_m_gt_n": lambda: synth.tiny(90, 35, 900, seed=5),
    "long_rows": long_rows_problem,
    "powerlaw": lambda: synth.netflix_shape(scale=0.03),
}
_cache = {}


def case(name):
    if name not in _cache:
        _cache[name] = CASES[name]()
    return _cache[name]


# ----------------------------------------------------------------------------- primitives

@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("k", [1, 5, 16, 17, 64, 80, 128, 129, 256])
def test_sddmm_parity(name, k):
    """k > 128 runs 16-lane groups (FP64 rows of more than 8 cache lines)."""
    p = case(name)
    print("sddmm", name, p.m, p.n, p.nnz, "k", k, flush=True)
    dp = to_dev(p, k_cap=128 if k <= 128 else 256)
    ld = bmg.round_ld(k)
    W, H = factors(p, k, ld, seed=k)
    R, hs = dp.bmg_sddmm(t(W), t(H), k)
    R = R.cpu().numpy()
    Ro = core.sddmm(p, W[:, :k], H[:, :k])
    bound = 4 * k * U * (core.sddmm(p, np.abs(W[:, :k]), np.abs(H[:, :k]), with_values=False)
                         + np.abs(p.val))
    assert np.all(np.abs(R - Ro) <= bound + 1e-300)
    assert math.isclose(hs, 0.5 * float(np.sum(Ro ** 2)), rel_tol=1e-12, abs_tol=1e-300)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("q", [1, 8, 33, 34, 65, 66, 130, 257])
@pytest.mark.parametrize("transpose", [False, True])
def test_spmm_parity(name, q, transpose):
    p = case(name)
    print("spmm", name, p.nnz, "q", q, "T", transpose, flush=True)
    dp = to_dev(p, k_cap=8)
    rng = np.random.default_rng(q)
    S = rng.standard_normal(p.nnz)
    ldq = bmg.round_ld(q)
    B = np.zeros((p.m if transpose else p.n, ldq))
    B[:, :q] = rng.standard_normal((B.shape[0], q))
    C = dp.bmg_spmm(t(S), t(B)[:, :].narrow(1, 0, ldq), transpose=transpose).cpu().numpy()[:, :q]
    if transpose:
        Co = core.spmm_t(p, S, B[:, :q])
        Cb = core.spmm_t(p, np.abs(S), np.abs(B[:, :q]))
        d = np.bincount(p.col, minlength=p.n)[:, None]
    else:
        Co = core.spmm(p, S, B[:, :q])
        Cb = core.spmm(p, np.abs(S), np.abs(B[:, :q]))
        d = np.diff(p.row_ptr)[:, None]
    assert np.all(np.abs(C - Co) <= 4 * np.maximum(d, 1) * U * Cb + 1e-300)


@pytest.mark.parametrize("name", ["tiny", "tall_m_gt_n", "long_rows", "powerlaw"])
@pytest.mark.parametrize("k", [6, 150])
def test_bm_epochs_parity(name, k):
    p = case(name)
    lam = 0.7
    kc = 16 if k <= 16 else 256
    dp = to_dev(p, k_cap=kc)
    ld = bmg.round_ld(kc)
    W, H = factors(p, k, ld, seed=3)
    Wd, Hd = t(W), t(H)
    Fbm = dp.bmg_bm_epochs(Wd, Hd, k, lam, epochs=2)
    # the library runs on the m <= n orientation (W step first there)
    tp = p.m > p.n
    q = core.transpose(p) if tp else p
    Wo, Ho = (H[:, :k], W[:, :k]) if tp else (W[:, :k], H[:, :k])
    for _ in range(2):
        Wo, Ho, _ = core.bm_epoch(q, Wo, Ho, lam)
    Fo = core.bm_objective(q, Wo, Ho, lam)
    if tp:
        Wo, Ho = Ho, Wo
    assert math.isclose(Fbm, Fo, rel_tol=1e-10)
    scale = max(np.abs(Wo).max(), np.abs(Ho).max())
    assert np.allclose(Wd.cpu().numpy()[:, :k], Wo, rtol=1e-8, atol=1e-9 * scale)
    assert np.allclose(Hd.cpu().numpy()[:, :k], Ho, rtol=1e-8, atol=1e-9 * scale)
    assert np.all(Wd.cpu().numpy()[:, k:] == 0)


@pytest.mark.parametrize("name", list(CASES))
def test_polymf_epochs_parity(name):
    """polyMF-SS BM epochs (column-pair BCD, exact quartic step) against the oracle's."""
    p = case(name)
    k, lam = 5, 0.7
    dp = to_dev(p, k_cap=8)
    W, H = factors(p, k, 8, seed=21)
    Wd, Hd = t(W), t(H)
    F = dp.bmg_polymf_epochs(Wd, Hd, k, lam, epochs=2)
    Wo, Ho = W[:, :k], H[:, :k]
    for _ in range(2):
        Wo, Ho, _ = core.polymf_epoch(p, Wo, Ho, lam)
    Fo = core.bm_objective(p, Wo, Ho, lam)
    Wg, Hg = Wd.cpu().numpy()[:, :k], Hd.cpu().numpy()[:, :k]
    print("polymf", name, F, Fo, flush=True)
    assert math.isclose(F, Fo, rel_tol=1e-10)
    sw, sh = np.abs(Wo).max(), np.abs(Ho).max()
    assert np.allclose(Wg, Wo, rtol=0, atol=1e-8 * sw) and np.allclose(Hg, Ho, rtol=0, atol=1e-8 * sh)


@pytest.mark.parametrize("name", ["tiny", "tall_m_gt_n", "powerlaw"])
def test_objective_parity(name):
    p = case(name)
    k = 5
    dp = to_dev(p, k_cap=8)
    W, H = factors(p, k, 8, seed=11)
    F = dp.bmg_objective(t(W), t(H), k, 0.9)
    assert math.isclose(F, core.objective(p, W[:, :k], H[:, :k], 0.9), rel_tol=1e-11)


@pytest.mark.parametrize("name", ["tiny", "tall_m_gt_n", "long_rows", "powerlaw"])
def test_objective_residual_parity(name):
    """bmg_objective's optional residual: the relative optimality residual of
    reading R1 at X = W H^T from one PG step at the default settings (alpha 1.99,
    seed 0, subspace tolerance 1e-12, at most 50 iterations), against the
    oracle's PG step from the same point; W and H are left untouched."""
    p = case(name)
    k, lam = 4, 0.4
    dp = to_dev(p, k_cap=32)
    W, H = factors(p, k, 32, seed=5)
    Wd, Hd = t(W), t(H)
    F, res = dp.bmg_objective(Wd, Hd, k, lam, residual=True)
    _, _, reso = core.prox_step_standalone(p, W[:, :k], H[:, :k], lam, 1.99, seed=0, tau=1e-12,
                                           max_iter=50)
    print("objective residual", name, res, reso, flush=True)
    assert math.isclose(F, core.objective(p, W[:, :k], H[:, :k], lam), rel_tol=1e-11)
    assert math.isclose(res, reso, rel_tol=1e-5, abs_tol=1e-12)
    assert np.array_equal(Wd.cpu().numpy(), W) and np.array_equal(Hd.cpu().numpy(), H)


@pytest.mark.parametrize("name", ["tiny", "tall_m_gt_n", "long_rows", "powerlaw"])
def test_prox_step_parity(name):
    p = case(name)
    lam, alpha, k = 0.4, 1.99, 4
    dp = to_dev(p, k_cap=32)
    W, H = factors(p, k, 32, seed=5)
    Wd, Hd = t(W), t(H)
    kg, sig, res = dp.bmg_prox_step(Wd, Hd, k, lam=lam, alpha=alpha, seed=9, ssi_tol_floor=1e-13,
                                    ssi_max_iter=200)
    pr, ls, reso = core.prox_step_standalone(p, W[:, :k], H[:, :k], lam, alpha, seed=9, tau=1e-13,
                                             max_iter=200)
    assert kg == pr.k
    assert np.allclose(sig, pr.sigma, rtol=1e-8, atol=1e-10 * max(pr.sigma.max(initial=0), 1))
    Wg, Hg = Wd.cpu().numpy()[:, :kg], Hd.cpu().numpy()[:, :kg]
    d = math.sqrt(core.diff_fro2_factored(Wg, Hg, pr.W, pr.H))
    assert d <= 1e-7 * max(1.0, math.sqrt(core.fro2_factored(pr.W, pr.H)))
    assert math.isclose(res, reso, rel_tol=1e-5, abs_tol=1e-12)


@pytest.mark.parametrize("hp", [1, 2])
@pytest.mark.parametrize("name", ["tiny", "tall_m_gt_n", "long_rows", "powerlaw"])
def test_prox_step_parity_lmsvd_history(name, hp):
    """Algorithm 2 with p_t = 1, 2 history blocks: the same prox output as the
    oracle's LmSVD with that history length."""
    p = case(name)
    lam, alpha, k = 0.4, 1.99, 4
    dp = to_dev(p, k_cap=32, lmsvd_p=hp)
    W, H = factors(p, k, 32, seed=5)
    Wd, Hd = t(W), t(H)
    kg, sig, res = dp.bmg_prox_step(Wd, Hd, k, lam=lam, alpha=alpha, seed=9, ssi_tol_floor=1e-13,
                                    ssi_max_iter=200, lmsvd_p=hp)
    pr, ls, reso = core.prox_step_standalone(p, W[:, :k], H[:, :k], lam, alpha, seed=9, tau=1e-13,
                                             max_iter=200, p=hp)
    print("prox history", name, hp, kg, pr.k, ls.iters, flush=True)
    assert kg == pr.k
    assert np.allclose(sig, pr.sigma, rtol=1e-8, atol=1e-10 * max(pr.sigma.max(initial=0), 1))
    Wg, Hg = Wd.cpu().numpy()[:, :kg], Hd.cpu().numpy()[:, :kg]
    d = math.sqrt(core.diff_fro2_factored(Wg, Hg, pr.W, pr.H))
    assert d <= 1e-7 * max(1.0, math.sqrt(core.fro2_factored(pr.W, pr.H)))
    assert math.isclose(res, reso, rel_tol=1e-5, abs_tol=1e-12)


# ----------------------------------------------------------------------------- solver

def solve_both(p, lam, k0, tol, k_cap=64, precision="fp64", seed=3, orc=None, bm_solver="polymf"):
    dp = to_dev(p, k_cap=k_cap, precision=precision)
    W, H, k, r = dp.bmg_solve(lam=lam, k_init=k0, tol=tol, seed=seed, max_iter=3000, bm_solver=bm_solver)
    if orc is None:
        orc = core.solve(p, core.Options(lam=lam, k0=k0, tol=tol, seed=seed, max_iter=3000, bm_solver=bm_solver))
    return dp, W, H, k, r, orc


@pytest.mark.parametrize("shape", [(40, 60, 700), (60, 40, 700), (120, 200, 4000)])
def test_solve_parity_fp64(shape):
    """The steepest-descent BM solver (polyMF-SS, the default, has its own test below)."""
    m, n, nnz = shape
    p = synth.tiny(m, n, nnz, rank=3, lam=0.3, seed=m + n)
    dp, W, H, k, r, orc = solve_both(p, 0.3, 4, 1e-10, bm_solver="psd")
    print("solve", shape, r, orc.F, orc.k, orc.iters, flush=True)
    assert r["status"] == 0 and orc.converged
    assert math.isclose(r["F"], orc.F, rel_tol=1e-8)
    assert k == orc.k
    # the returned factors reproduce the reported objective (recomputed by the oracle)
    Fw = core.objective(p, W.cpu().numpy()[:, :k], H.cpu().numpy()[:, :k], 0.3)
    assert math.isclose(Fw, r["F"], rel_tol=1e-10)


@pytest.mark.parametrize("hp", [1, 2])
@pytest.mark.parametrize("shape", [(40, 60, 700), (60, 40, 700), (120, 200, 4000)])
def test_solve_parity_fp64_lmsvd_history(shape, hp):
    m, n, nnz = shape
    p = synth.tiny(m, n, nnz, rank=3, lam=0.3, seed=m + n)
    recs = []
    orc = core.solve(p, core.Options(lam=0.3, k0=4, tol=1e-10, seed=3, max_iter=3000, lmsvd_p=hp),
                     callback=recs.append)
    dp = to_dev(p, k_cap=64, lmsvd_p=hp)
    W, H, k, r = dp.bmg_solve(lam=0.3, k_init=4, tol=1e-10, seed=3, max_iter=3000, lmsvd_p=hp)
    print("solve history", shape, hp, r["ssi_iters"], sum(x.ssi_iters for x in recs), r["F"], orc.F,
          flush=True)
    assert r["status"] == 0 and orc.converged
    assert math.isclose(r["F"], orc.F, rel_tol=1e-8)
    assert k == orc.k
    Fw = core.objective(p, W.cpu().numpy()[:, :k], H.cpu().numpy()[:, :k], 0.3)
    assert math.isclose(Fw, r["F"], rel_tol=1e-10)


@pytest.mark.parametrize("precision,bar", [("fp32", 1e-5), ("bf16", 1e-3)])
def test_solve_lmsvd_history_reduced_precision(precision, bar):
    p = synth.tiny(150, 220, 5000, rank=3, lam=0.3, seed=31)
    dp = to_dev(p, k_cap=64, precision=precision, lmsvd_p=1)
    W, H, k, r = dp.bmg_solve(lam=0.3, k_init=4, tol=1e-6 if precision == "fp32" else 1e-5, seed=3,
                              max_iter=600, lmsvd_p=1)
    Fw = core.objective(p, W.cpu().numpy()[:, :k], H.cpu().numpy()[:, :k], 0.3)
    Fstar = core.solve(p, core.Options(lam=0.3, k0=4, tol=1e-11, seed=3)).F
    print("history", precision, r["status"], r["iters"], r["ssi_iters"], Fw, Fstar, flush=True)
    assert r["status"] == 0
    assert abs(Fw - Fstar) <= bar * Fstar


@pytest.mark.parametrize("shape", [(40, 60, 700), (60, 40, 700), (120, 200, 4000), (300, 500, 30000)])
def test_solve_parity_fp64_sparsa(shape):
    """SpaRSA step rule (BB step + backtracking on eq. back) against the oracle's."""
    m, n, nnz = shape
    lam = 1.0 if nnz > 10000 else 0.3
    p = synth.tiny(m, n, nnz, rank=3 if nnz < 10000 else 8, lam=lam, seed=m + n)
    recs = []
    orc = core.solve(p, core.Options(lam=lam, k0=4, tol=1e-10, seed=3, max_iter=3000,
                                     step_rule="sparsa"), callback=recs.append)
    dp = to_dev(p, k_cap=128, sparsa=True)
    W, H, k, r = dp.bmg_solve(lam=lam, k_init=4, tol=1e-10, seed=3, max_iter=3000, step_rule="sparsa")
    print("sparsa", shape, r["iters"], orc.iters, r["pg_trials"], sum(x.trials for x in recs),
          r["alpha_last"], recs[-1].alpha, r["F"], orc.F, flush=True)
    assert r["status"] == 0 and orc.converged
    assert math.isclose(r["F"], orc.F, rel_tol=1e-8)
    assert k == orc.k
    assert r["pg_trials"] >= r["iters"]
    Fw = core.objective(p, W.cpu().numpy()[:, :k], H.cpu().numpy()[:, :k], lam)
    assert math.isclose(Fw, r["F"], rel_tol=1e-10)


def test_sparsa_with_equal_bounds_is_the_fixed_step_bitwise():
    p = synth.tiny(120, 200, 4000, rank=3, lam=0.3, seed=320)
    outs = []
    for kw in ({}, {"step_rule": "sparsa", "alpha_min": 1.99, "alpha_max": 1.99}):
        W, H, k, r = to_dev(p, k_cap=64, sparsa=True).bmg_solve(lam=0.3, k_init=4, tol=1e-10, seed=3, **kw)
        outs.append((W.cpu().numpy(), H.cpu().numpy(), k, r["iters"], r["pg_trials"]))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    assert outs[0][2:] == outs[1][2:] and outs[1][4] == outs[1][3]


def test_solve_sparsa_fp32_objective_error():
    p = synth.tiny(150, 220, 5000, rank=3, lam=0.3, seed=31)
    dp = to_dev(p, k_cap=64, precision="fp32", sparsa=True)
    W, H, k, r = dp.bmg_solve(lam=0.3, k_init=4, tol=1e-6, seed=3, max_iter=600, step_rule="sparsa")
    Fw = core.objective(p, W.cpu().numpy()[:, :k], H.cpu().numpy()[:, :k], 0.3)
    Fstar = core.solve(p, core.Options(lam=0.3, k0=4, tol=1e-11, seed=3)).F
    print("sparsa fp32", r["status"], r["iters"], r["pg_trials"], Fw, Fstar, flush=True)
    assert r["status"] == 0
    assert abs(Fw - Fstar) <= 1e-5 * Fstar


@pytest.mark.parametrize("shape", [(40, 60, 700), (60, 40, 700), (120, 200, 4000)])
def test_solve_parity_fp64_polymf(shape):
    m, n, nnz = shape
    p = synth.tiny(m, n, nnz, rank=3, lam=0.3, seed=m + n)
    orc = core.solve(p, core.Options(lam=0.3, k0=4, tol=1e-10, seed=3, max_iter=3000, bm_solver="polymf"))
    dp = to_dev(p, k_cap=64)
    W, H, k, r = dp.bmg_solve(lam=0.3, k_init=4, tol=1e-10, seed=3, max_iter=3000, bm_solver="polymf")
    print("solve polymf", shape, r["iters"], orc.iters, r["F"], orc.F, flush=True)
    assert r["status"] == 0 and orc.converged
    assert math.isclose(r["F"], orc.F, rel_tol=1e-8)
    assert k == orc.k
    Fw = core.objective(p, W.cpu().numpy()[:, :k], H.cpu().numpy()[:, :k], 0.3)
    assert math.isclose(Fw, r["F"], rel_tol=1e-10)


@pytest.mark.parametrize("precision,bar", [("fp32", 1e-5), ("bf16", 1e-3)])
def test_solve_polymf_reduced_precision(precision, bar):
    p = synth.tiny(150, 220, 5000, rank=3, lam=0.3, seed=31)
    dp = to_dev(p, k_cap=64, precision=precision)
    W, H, k, r = dp.bmg_solve(lam=0.3, k_init=4, tol=1e-6 if precision == "fp32" else 1e-5, seed=3,
                              max_iter=600, bm_solver="polymf")
    Fw = core.objective(p, W.cpu().numpy()[:, :k], H.cpu().numpy()[:, :k], 0.3)
    Fstar = core.solve(p, core.Options(lam=0.3, k0=4, tol=1e-11, seed=3)).F
    print("polymf", precision, r["status"], r["iters"], Fw, Fstar, flush=True)
    assert r["status"] == 0
    assert abs(Fw - Fstar) <= bar * Fstar


@pytest.mark.parametrize("shape", [(60, 40, 700), (120, 200, 4000)])
def test_solve_parity_all_variants_together(shape):
    """polyMF-SS BM phase, SpaRSA step rule and LmSVD with one history block in
    one solve, against the oracle with the same options."""
    m, n, nnz = shape
    p = synth.tiny(m, n, nnz, rank=3, lam=0.3, seed=m + n + 1)
    orc = core.solve(p, core.Options(lam=0.3, k0=4, tol=1e-10, seed=5, max_iter=3000, bm_solver="polymf",
                                     step_rule="sparsa", lmsvd_p=1))
    dp = to_dev(p, k_cap=64, lmsvd_p=1, sparsa=True)
    W, H, k, r = dp.bmg_solve(lam=0.3, k_init=4, tol=1e-10, seed=5, max_iter=3000, bm_solver="polymf",
                              step_rule="sparsa", lmsvd_p=1)
    print("all variants", shape, r["iters"], orc.iters, r["pg_trials"], r["F"], orc.F, flush=True)
    assert r["status"] == 0 and orc.converged
    assert math.isclose(r["F"], orc.F, rel_tol=1e-8)
    assert k == orc.k


def test_solve_full_omega_closed_form():
    m, n, lam = 30, 45, 1.5
    p = synth.tiny(m, n, m * n, rank=4, seed=12)
    A, _ = dense.to_dense(p)
    dp = to_dev(p, k_cap=32)
    W, H, k, r = dp.bmg_solve(lam=lam, k_init=4, tol=1e-12, seed=1)
    X = W.cpu().numpy()[:, :k] @ H.cpu().numpy()[:, :k].T
    assert np.allclose(X, dense.prox_nuclear(A, lam), atol=1e-8)


def test_solve_zero_solution_and_empty():
    p = synth.tiny(20, 30, 200, seed=6)
    A, _ = dense.to_dense(p)
    lam = 1.01 * np.linalg.svd(A, compute_uv=False)[0]
    W, H, k, r = to_dev(p, 16).bmg_solve(lam=lam, k_init=4, tol=1e-10)
    assert k == 0 and math.isclose(r["F"], 0.5 * float(np.sum(p.val ** 2)), rel_tol=1e-13)
    pe = synth.tiny(8, 9, 0)
    W, H, k, r = to_dev(pe, 8).bmg_solve(lam=0.1, k_init=3, tol=1e-10)
    assert k == 0 and r["F"] == 0.0


def test_solve_small_uniform_matches_golden(golden_dir):
    """1000 x 1500, |Omega| = 50,000, lambda = 0.5, k0 = 8: F within 1e-8 of the
    oracle optimum stored in tests/golden (itself certified by a duality gap)."""
    g = json.load(open(os.path.join(golden_dir, "small_uniform.json")))
    p = synth.small_uniform()
    dp = to_dev(p, k_cap=128)
    W, H, k, r = dp.bmg_solve(lam=p.lam, k_init=p.k0, tol=1e-10, seed=11, max_iter=3000)
    print("small_uniform", r, flush=True)
    assert r["status"] == 0
    assert abs(r["F"] - g["F"]) <= 1e-8 * g["F"]
    assert k == g["rank"]


def test_netflix_quarter_solves_match_the_certified_optimum(golden_dir):
    """Netflix-shaped generator at scale 0.25 (4,442 x 120,047, |Omega| = 6.25e6,
    power-law degrees), lambda = 300, k0 = 16: the FP64, FP32 and BF16 solves
    against the oracle optimum stored in tests/golden (its duality gap certifies
    it to 2e-10 relative): objective error <= 1e-8 (FP64), 1e-5 (FP32) and 1e-3
    (BF16, FP64 refresh every 5 iterations), same rank."""
    g = json.load(open(os.path.join(golden_dir, "netflix_quarter_lam300.json")))
    assert g["dual_gap"] <= 1e-9 * g["F"]
    p = synth.netflix_shape(scale=0.25)
    assert p.name == g["problem"]
    evaluator = to_dev(p, k_cap=64)
    for prec, tol, bar in (("fp64", 1e-8, 1e-8), ("fp32", 1e-6, 1e-5), ("bf16", 1e-5, 1e-3)):
        dp = to_dev(p, k_cap=64, precision=prec)
        W, H, k, r = dp.bmg_solve(lam=g["lam"], k_init=g["k0"], tol=tol, seed=3, max_iter=1000)
        F64 = evaluator.bmg_objective(W, H, k, g["lam"])
        err = abs(F64 - g["F"]) / g["F"]
        print("netflix x0.25", prec, r["status"], r["iters"], k, r["F"], F64, err, flush=True)
        assert r["status"] == 0 and k == g["rank"]
        assert err <= bar
        del dp


def test_powerlaw_solve_three_iterations_matches_oracle():
    """The Netflix-shaped generator at scale 0.03 (power-law rows and columns,
    fully dense rows): three outer iterations from the same seed on both sides,
    objective and rank after each solve's last iteration."""
    p = case("powerlaw")
    lam = 20.0
    dp = to_dev(p, k_cap=64)
    W, H, k, r = dp.bmg_solve(lam=lam, k_init=8, tol=0.0, seed=4, max_iter=3)
    orc = core.solve(p, core.Options(lam=lam, k0=8, tol=0.0, seed=4, max_iter=3))
    print("powerlaw 3 iterations", r["F"], orc.F, k, orc.k, r["residual"], orc.residual, flush=True)
    assert r["iters"] == 3 and orc.iters == 3
    assert k == orc.k
    assert math.isclose(r["F"], orc.F, rel_tol=1e-8)
    Fw = core.objective(p, W.cpu().numpy()[:, :k], H.cpu().numpy()[:, :k], lam)
    assert math.isclose(Fw, r["F"], rel_tol=1e-10)


def test_solve_fp32_objective_error():
    p = synth.tiny(150, 220, 5000, rank=3, lam=0.3, seed=31)
    dp, W, H, k, r, orc = solve_both(p, 0.3, 4, 1e-6, precision="fp32")
    Fw = core.objective(p, W.cpu().numpy()[:, :k], H.cpu().numpy()[:, :k], 0.3)
    Fstar = core.solve(p, core.Options(lam=0.3, k0=4, tol=1e-11, seed=3)).F
    print("fp32", r, Fw, Fstar, flush=True)
    assert abs(Fw - Fstar) <= 1e-5 * Fstar


@pytest.mark.parametrize("refresh", [2, 5])
def test_solve_bf16_objective_error(refresh):
    """BF16 gathers, FP32 accumulation, FP64 residual/objective refresh every
    `refresh` outer iterations (those skip the BM phase and gather FP32 in the
    PG step): objective within 1e-3 of the FP64 optimum."""
    p = synth.tiny(150, 220, 5000, rank=3, lam=0.3, seed=31)
    dp = to_dev(p, k_cap=64, precision="bf16")
    W, H, k, r = dp.bmg_solve(lam=0.3, k_init=4, tol=1e-5, seed=3, max_iter=600,
                              refresh_every=refresh)
    Fw = core.objective(p, W.cpu().numpy()[:, :k], H.cpu().numpy()[:, :k], 0.3)
    Fstar = core.solve(p, core.Options(lam=0.3, k0=4, tol=1e-11, seed=3)).F
    print("bf16", refresh, r["status"], r["iters"], r["residual"], Fw, Fstar, (Fw - Fstar) / Fstar,
          flush=True)
    assert r["status"] == 0
    assert abs(Fw - Fstar) <= 1e-3 * Fstar
    # the reported F is the FP64 objective of the FP32 master factors
    assert math.isclose(r["F"], Fw, rel_tol=1e-6)


def test_solve_is_bitwise_deterministic():
    p = synth.netflix_shape(scale=0.02)
    outs = []
    for _ in range(2):
        dp = to_dev(p, k_cap=32)
        W, H, k, r = dp.bmg_solve(lam=20.0, k_init=4, tol=1e-5, max_iter=5, seed=2)
        outs.append((W.cpu().numpy(), H.cpu().numpy(), r["F"]))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    assert outs[0][2] == outs[1][2]


# ----------------------------------------------------------------------------- errors

def test_invalid_inputs_are_rejected():
    p = synth.tiny(6, 7, 20)
    bad = p.col.copy(); bad[1], bad[2] = bad[2], bad[1]     # unsorted within a row? ensure same row
    rows = p.rows()
    if rows[1] == rows[2]:
        with pytest.raises(bmg.BmgError, match="BMG_EINVAL"):
            bmg.Problem.from_host(p.row_ptr, bad, p.val, p.m, p.n, device=DEV)
    oob = p.col.copy(); oob[0] = p.n
    with pytest.raises(bmg.BmgError, match="BMG_EINVAL"):
        bmg.Problem.from_host(p.row_ptr, oob, p.val, p.m, p.n, device=DEV)
    nanv = p.val.copy(); nanv[3] = np.nan
    with pytest.raises(bmg.BmgError, match="BMG_ENONFINITE"):
        bmg.Problem.from_host(p.row_ptr, p.col, nanv, p.m, p.n, device=DEV)
    dp = to_dev(p, k_cap=8)
    with pytest.raises(bmg.BmgError, match="BMG_EINVAL"):
        dp.bmg_solve(lam=-1.0)
    for hp in (-1, 5):
        with pytest.raises(bmg.BmgError, match="BMG_EINVAL"):
            dp.bmg_solve(lam=0.1, lmsvd_p=hp)
    with pytest.raises(bmg.BmgError, match="BMG_EINVAL"):
        dp.bmg_polymf_epochs(t(np.zeros((6, 8))), t(np.zeros((7, 8))), 2, -1.0)
    for kw in ({"bm_solver": 2}, {"step_rule": 2}, {"step_rule": "sparsa", "sparsa_beta": 1.0},
               {"step_rule": "sparsa", "alpha_min": 5.0, "alpha_max": 2.0},
               {"step_rule": "sparsa", "sparsa_delta": 0.0}):
        with pytest.raises(bmg.BmgError, match="BMG_EINVAL"):
            dp.bmg_solve(lam=0.1, **kw)
    # variants the workspace was not sized for are refused, nothing is allocated
    with pytest.raises(bmg.BmgError, match="BMG_ENOMEM"):
        dp.bmg_solve(lam=0.1, lmsvd_p=1)
    with pytest.raises(bmg.BmgError, match="BMG_ENOMEM"):
        dp.bmg_solve(lam=0.1, step_rule="sparsa")
    with pytest.raises(bmg.BmgError, match="BMG_ENOMEM"):
        to_dev(p, k_cap=8, lmsvd_p=1).bmg_solve(lam=0.1, lmsvd_p=2)


# ----------------------------------------------------------------------------- full size, sampled

def test_netflix_shape_full_size_sampled_rows():
    """17,770 x 480,189, |Omega| = 1e8 (the benchmark's workload): the sampled
    residual and both gradient products on sampled rows / columns against the
    oracle evaluated on those rows only."""
    p = synth.netflix_shape()
    k, lam = 16, 20.0
    dp = to_dev(p, k_cap=16)
    W, H = factors(p, k, 16, seed=7)
    W *= 0.3; H *= 0.3
    R, hs = dp.bmg_sddmm(t(W), t(H), k)
    rows = np.random.default_rng(1).choice(p.m, 64, replace=False)
    rows = np.union1d(rows, np.argsort(np.diff(p.row_ptr))[-4:])     # include dense rows
    Rg = R.cpu().numpy()
    for i in rows:
        a, b = p.row_ptr[i], p.row_ptr[i + 1]
        ro = W[i, :k] @ H[p.col[a:b], :k].T - p.val[a:b]
        assert np.allclose(Rg[a:b], ro, rtol=1e-12, atol=1e-12)
    # gradient products R H and R^T W on sampled rows / columns
    GW = dp.bmg_spmm(R, t(H)).cpu().numpy()
    for i in rows[:16]:
        a, b = p.row_ptr[i], p.row_ptr[i + 1]
        assert np.allclose(GW[i, :k], Rg[a:b] @ H[p.col[a:b], :k], rtol=1e-10, atol=1e-9)
    GH = dp.bmg_spmm(R, t(W), transpose=True).cpu().numpy()
    cols = np.random.default_rng(2).choice(p.n, 16, replace=False)
    prow = p.rows()
    for j in cols:
        sel = np.nonzero(p.col == j)[0]
        assert np.allclose(GH[j, :k], Rg[sel] @ W[prow[sel], :k], rtol=1e-10, atol=1e-9)


def test_netflix_shape_full_size_polymf_block():
    """One polyMF-SS block (an epoch at k = 1) on the full 1e8-entry workload:
    both direction passes (long rows cut into pieces), the quartic sums and the
    step, against the oracle's block on the whole problem."""
    p = synth.netflix_shape()
    lam = 20.0
    dp = to_dev(p, k_cap=8)
    W, H = factors(p, 1, 8, seed=17)
    W *= 0.3; H *= 0.3
    Wd, Hd = t(W), t(H)
    F = dp.bmg_polymf_epochs(Wd, Hd, 1, lam, epochs=1)
    Wo, Ho, Ro, step = core.polymf_block(p, W[:, :1], H[:, :1], 0, lam, core.sddmm(p, W[:, :1], H[:, :1]))
    del Ro
    Fo = core.bm_objective(p, Wo, Ho, lam)
    print("polymf full size: step", step, "F", F, Fo, flush=True)
    assert step > 0 and math.isclose(F, Fo, rel_tol=1e-10)
    Wg, Hg = Wd.cpu().numpy()[:, :1], Hd.cpu().numpy()[:, :1]
    assert np.allclose(Wg, Wo, rtol=0, atol=1e-9 * np.abs(Wo).max())
    assert np.allclose(Hg, Ho, rtol=0, atol=1e-9 * np.abs(Ho).max())


def test_yahoo_shape_full_size_sampled_rows_and_fp32_step():
    """624,961 x 1,000,990, |Omega| = 2.5e8 (capped power law, exponent 1.1):
    FP64 sampled residual and both sparse products on sampled rows / columns
    against the oracle on those rows only (both orientations cut long rows at
    column ranges), then one FP32 outer iteration whose reported objective must
    match the oracle's FP64 objective at the returned factors."""
    p = synth.yahoo_shape()
    k = 8
    dp = to_dev(p, k_cap=16)
    W, H = factors(p, k, 16, seed=9)
    W *= 0.3; H *= 0.3
    R, _ = dp.bmg_sddmm(t(W), t(H), k)
    Rg = R.cpu().numpy()
    L = np.diff(p.row_ptr)
    rows = np.union1d(np.random.default_rng(3).choice(p.m, 32, replace=False), np.argsort(L)[-4:])
    for i in rows:
        a, b = p.row_ptr[i], p.row_ptr[i + 1]
        ro = W[i, :k] @ H[p.col[a:b], :k].T - p.val[a:b]
        assert np.allclose(Rg[a:b], ro, rtol=1e-12, atol=1e-12)
    GW = dp.bmg_spmm(R, t(H)).cpu().numpy()
    for i in rows:
        a, b = p.row_ptr[i], p.row_ptr[i + 1]
        assert np.allclose(GW[i, :k], Rg[a:b] @ H[p.col[a:b], :k], rtol=1e-10, atol=1e-9)
    GH = dp.bmg_spmm(R, t(W), transpose=True).cpu().numpy()
    C = np.bincount(p.col, minlength=p.n)
    cols = np.union1d(np.random.default_rng(4).choice(p.n, 12, replace=False), np.argsort(C)[-2:])
    sel = np.nonzero(np.isin(p.col, cols))[0]
    prow = np.searchsorted(p.row_ptr, sel, side="right") - 1
    for j in cols:
        s = p.col[sel] == j
        assert np.allclose(GH[j, :k], Rg[sel[s]] @ W[prow[s], :k], rtol=1e-10, atol=1e-9)
    del dp, R, Rg, GW, GH
    torch.cuda.empty_cache()
    # one outer iteration in FP32; F is reported in FP64 from the returned factors
    d32 = to_dev(p, k_cap=128, precision="fp32")   # one step can reach 2 k0 + 1 columns
    Wd, Hd, kk, r = d32.bmg_solve(lam=p.lam, k_init=p.k0, max_iter=1, tol=0.0, seed=5)
    Wn, Hn = Wd.cpu().numpy()[:, :kk], Hd.cpu().numpy()[:, :kk]
    F_orc = core.objective(p, Wn, Hn, p.lam)
    assert kk >= 1
    assert abs(r["F"] - F_orc) <= 1e-5 * abs(F_orc), (r["F"], F_orc)
