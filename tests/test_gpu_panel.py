"""Dense-row panel (bmg_options.dense_rows): the rows of Omega at least that
dense leave the gather passes and go through the dense panel kernels (solves
with the steepest-descent BM solver: polyMF-SS, the default, and SpaRSA read
the stored residual entry by entry and run without the panel).  The
oracle knows nothing of panels, so every result is held to the same bars as
without one: BM epochs, objective, prox step and solves against the oracle, and
the panel path against the plain path of the library on the full-size
Netflix-shaped step.

Bars as in test_gpu_parity: BM objective and factors to 1e-10 / 1e-8, objective
to 1e-11, prox singular values to 1e-8, solve objective 1e-8 (FP64) and 1e-5
(FP32) with the same rank."""
import math

import numpy as np
import pytest
import torch

import paper_2204_14067_amd as bmg
import synth
from oracle import core

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def dense_rows_problem(m, n, dense, frac, nnz_sparse, seed, rank=3, lam=0.5):
    """Rows `dense` observe a fraction `frac` of the columns, the others share
    nnz_sparse uniform entries; values from a rank-`rank` truth + noise."""
    rng = np.random.default_rng(seed)
    cols = []
    sparse_rows = [i for i in range(m) if i not in dense]
    per = np.bincount(rng.choice(len(sparse_rows), nnz_sparse), minlength=len(sparse_rows))
    cnt = dict(zip(sparse_rows, per))
    for i in range(m):
        if i in dense:
            c = np.sort(rng.choice(n, int(frac * n), replace=False))
        else:
            c = np.sort(rng.choice(n, min(n, int(cnt[i])), replace=False))
        cols.append(c.astype(np.int32))
    row_ptr = np.zeros(m + 1, np.int64)
    row_ptr[1:] = np.cumsum([len(c) for c in cols])
    col = np.concatenate(cols)
    val, _, _ = synth.values(m, n, row_ptr, col, rank, 1.0 / math.sqrt(rank), 0.01, seed=seed + 1)
    return synth.Problem("dense_rows_%dx%d_nnz%d" % (m, n, len(col)), m, n, row_ptr, col, val, lam, 4)


def transposed(p):
    q = core.transpose(p)
    return synth.Problem(p.name + "_T", q.m, q.n, q.row_ptr, q.col, q.val, p.lam, p.k0)


CASES = {
    "mixed": lambda: dense_rows_problem(60, 400, (0, 7, 33), 0.9, 3000, seed=5),
    "mixed_m_gt_n": lambda: transposed(dense_rows_problem(50, 300, (3, 20, 21, 49), 0.6, 2500, seed=6)),
    "all_dense": lambda: dense_rows_problem(12, 900, tuple(range(12)), 0.35, 0, seed=7),
    "powerlaw": lambda: synth.netflix_shape(scale=0.03),
    # panels of 100 and 200 rows: several panel-row tiles per wave in the rows
    # product, and large LDS copies of the gathered rows in the columns product
    "tall_panel": lambda: dense_rows_problem(220, 700, tuple(range(0, 200, 2)), 0.4, 4000, seed=8),
    "taller_panel": lambda: dense_rows_problem(230, 500, tuple(range(200)), 0.3, 1500, seed=9),
}
_cache = {}


def case(name):
    if name not in _cache:
        _cache[name] = CASES[name]()
    return _cache[name]


def to_dev(p, k_cap=32, precision="fp64", dense_rows=0.25):
    return bmg.Problem.from_host(p.row_ptr, p.col, p.val, p.m, p.n, k_cap=k_cap, precision=precision,
                                 device=DEV, dense_rows=dense_rows)


def t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def factors(p, k, ld, seed):
    rng = np.random.default_rng(seed)
    W = np.zeros((p.m, ld)); H = np.zeros((p.n, ld))
    W[:, :k] = rng.standard_normal((p.m, k))
    H[:, :k] = rng.standard_normal((p.n, k))
    return W, H


def test_cases_have_dense_rows():
    for name in CASES:
        p = case(name)
        q = core.transpose(p) if p.m > p.n else p
        deg = np.diff(q.row_ptr)
        assert np.sum(deg >= 0.25 * q.n) >= 1, name
        print(name, p.m, p.n, p.nnz, "panel rows", int(np.sum(deg >= 0.25 * q.n)), flush=True)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("k", [3, 16, 33])
def test_panel_bm_epochs_parity(name, k):
    p = case(name)
    lam = 0.7
    dp = to_dev(p, k_cap=48)
    ld = bmg.round_ld(48)
    W, H = factors(p, k, ld, seed=3)
    Wd, Hd = t(W), t(H)
    Fbm = dp.bmg_bm_epochs(Wd, Hd, k, lam, epochs=2)
    tp = p.m > p.n
    q = core.transpose(p) if tp else p
    Wo, Ho = (H[:, :k], W[:, :k]) if tp else (W[:, :k], H[:, :k])
    for _ in range(2):
        Wo, Ho, _ = core.bm_epoch(q, Wo, Ho, lam)
    Fo = core.bm_objective(q, Wo, Ho, lam)
    if tp:
        Wo, Ho = Ho, Wo
    print("panel bm", name, k, Fbm, Fo, flush=True)
    assert math.isclose(Fbm, Fo, rel_tol=1e-10)
    scale = max(np.abs(Wo).max(), np.abs(Ho).max())
    assert np.allclose(Wd.cpu().numpy()[:, :k], Wo, rtol=1e-8, atol=1e-9 * scale)
    assert np.allclose(Hd.cpu().numpy()[:, :k], Ho, rtol=1e-8, atol=1e-9 * scale)


@pytest.mark.parametrize("name", ["tall_panel", "taller_panel"])
@pytest.mark.parametrize("k", [50, 70, 100])
def test_panel_bm_epochs_parity_wide(name, k):
    """Widths of 4 to 7 output tiles of 16 (the columns product falls back to
    its register-staged form beyond 5) on panels of 100 and 200 rows."""
    p = case(name)
    lam = 0.7
    dp = to_dev(p, k_cap=112)
    ld = bmg.round_ld(112)
    W, H = factors(p, k, ld, seed=4)
    Wd, Hd = t(W), t(H)
    Fbm = dp.bmg_bm_epochs(Wd, Hd, k, lam, epochs=2)
    Wo, Ho = W[:, :k], H[:, :k]
    for _ in range(2):
        Wo, Ho, _ = core.bm_epoch(p, Wo, Ho, lam)
    Fo = core.bm_objective(p, Wo, Ho, lam)
    print("panel bm wide", name, k, Fbm, Fo, flush=True)
    assert math.isclose(Fbm, Fo, rel_tol=1e-10)
    scale = max(np.abs(Wo).max(), np.abs(Ho).max())
    assert np.allclose(Wd.cpu().numpy()[:, :k], Wo, rtol=1e-8, atol=1e-9 * scale)
    assert np.allclose(Hd.cpu().numpy()[:, :k], Ho, rtol=1e-8, atol=1e-9 * scale)


@pytest.mark.parametrize("name", list(CASES))
def test_panel_objective_parity(name):
    p = case(name)
    k = 5
    dp = to_dev(p, k_cap=8)
    W, H = factors(p, k, 8, seed=11)
    F = dp.bmg_objective(t(W), t(H), k, 0.9)
    assert math.isclose(F, core.objective(p, W[:, :k], H[:, :k], 0.9), rel_tol=1e-11)


@pytest.mark.parametrize("name", list(CASES))
def test_panel_prox_step_parity(name):
    p = case(name)
    lam, alpha, k = 0.4, 1.99, 4
    dp = to_dev(p, k_cap=32)
    W, H = factors(p, k, 32, seed=5)
    Wd, Hd = t(W), t(H)
    kg, sig, res = dp.bmg_prox_step(Wd, Hd, k, lam=lam, alpha=alpha, seed=9, ssi_tol_floor=1e-13,
                                    ssi_max_iter=200)
    pr, ls, reso = core.prox_step_standalone(p, W[:, :k], H[:, :k], lam, alpha, seed=9, tau=1e-13,
                                             max_iter=200)
    print("panel prox", name, kg, pr.k, flush=True)
    assert kg == pr.k
    assert np.allclose(sig, pr.sigma, rtol=1e-8, atol=1e-10 * max(pr.sigma.max(initial=0), 1))
    Wg, Hg = Wd.cpu().numpy()[:, :kg], Hd.cpu().numpy()[:, :kg]
    d = math.sqrt(core.diff_fro2_factored(Wg, Hg, pr.W, pr.H))
    assert d <= 1e-7 * max(1.0, math.sqrt(core.fro2_factored(pr.W, pr.H)))
    assert math.isclose(res, reso, rel_tol=1e-5, abs_tol=1e-12)


@pytest.mark.parametrize("name", ["mixed", "mixed_m_gt_n", "all_dense"])
def test_panel_solve_parity_fp64(name):
    p = case(name)
    lam = 0.5
    dp = to_dev(p, k_cap=64)
    W, H, k, r = dp.bmg_solve(lam=lam, k_init=4, tol=1e-10, seed=3, max_iter=3000, bm_solver="psd")
    orc = core.solve(p, core.Options(lam=lam, k0=4, tol=1e-10, seed=3, max_iter=3000, bm_solver="psd"))
    print("panel solve", name, r["iters"], orc.iters, k, orc.k, r["F"], orc.F, flush=True)
    assert r["status"] == 0 and orc.converged
    assert math.isclose(r["F"], orc.F, rel_tol=1e-8)
    assert k == orc.k
    Fw = core.objective(p, W.cpu().numpy()[:, :k], H.cpu().numpy()[:, :k], lam)
    assert math.isclose(Fw, r["F"], rel_tol=1e-10)


def test_panel_solve_fp32_objective_error():
    p = case("mixed")
    lam = 0.5
    dp = to_dev(p, k_cap=64, precision="fp32")
    W, H, k, r = dp.bmg_solve(lam=lam, k_init=4, tol=1e-6, seed=3, max_iter=3000, bm_solver="psd")
    Fw = core.objective(p, W.cpu().numpy()[:, :k], H.cpu().numpy()[:, :k], lam)
    Fstar = core.solve(p, core.Options(lam=lam, k0=4, tol=1e-11, seed=3, max_iter=3000)).F
    print("panel fp32", r["status"], r["iters"], Fw, Fstar, flush=True)
    assert r["status"] == 0
    assert abs(Fw - Fstar) <= 1e-5 * Fstar


def test_panel_solve_is_bitwise_deterministic_and_matches_plain_path():
    p = case("powerlaw")
    outs = []
    for dr in (0.25, 0.25, 0.0):
        dp = to_dev(p, k_cap=64, dense_rows=dr)
        W, H, k, r = dp.bmg_solve(lam=20.0, k_init=8, tol=1e-7, max_iter=200, seed=2, bm_solver="psd")
        outs.append((W.cpu().numpy(), H.cpu().numpy(), r["F"], k, r["iters"]))
        print("powerlaw dense_rows", dr, k, r["F"], r["iters"], flush=True)
    assert np.array_equal(outs[0][0], outs[1][0]) and outs[0][2] == outs[1][2]
    assert outs[0][3] == outs[2][3]
    assert math.isclose(outs[0][2], outs[2][2], rel_tol=1e-9)


def test_panel_variants_switch_it_off():
    """polyMF-SS and SpaRSA read the stored residual entry by entry: on a problem
    with a panel they run the plain passes and match the oracle."""
    p = case("mixed")
    lam = 0.5
    dp = bmg.Problem.from_host(p.row_ptr, p.col, p.val, p.m, p.n, k_cap=64, device=DEV, dense_rows=0.25,
                               sparsa=True)
    for kw in ({"bm_solver": "polymf"}, {"step_rule": "sparsa"}):
        W, H, k, r = dp.bmg_solve(lam=lam, k_init=4, tol=1e-10, seed=3, max_iter=3000, **kw)
        orc = core.solve(p, core.Options(lam=lam, k0=4, tol=1e-10, seed=3, max_iter=3000, **kw))
        assert r["status"] == 0 and k == orc.k
        assert math.isclose(r["F"], orc.F, rel_tol=1e-8)


def test_netflix_shape_full_size_panel_step_matches_plain_path():
    """The benchmark step on the full 1e8-entry Netflix-shaped workload (46 fully
    dense rows; rows at >= 25% density hold 45% of the entries): with the panel
    and without it, the same rank and objective after the step."""
    p = synth.netflix_shape()
    res = {}
    for dr in (0.25, 0.0):
        dp = to_dev(p, k_cap=64, dense_rows=dr)
        W, H = dp.zeros_factors()
        _, _, k, r = dp.bmg_solve(W, H, lam=20.0, k_init=16, max_iter=1, tol=0.0, seed=1003, bm_solver="psd")
        res[dr] = (k, r["F"], r["ssi_iters"])
        print("netflix step dense_rows", dr, res[dr], flush=True)
        del dp, W, H
        torch.cuda.empty_cache()
    assert res[0.25][0] == res[0.0][0] and res[0.25][2] == res[0.0][2]
    assert math.isclose(res[0.25][1], res[0.0][1], rel_tol=1e-9)
