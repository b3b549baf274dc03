"""Pins of the CPU oracle against facts fixed by the paper and by mathematics
(CPU only).  A plausible slip anywhere in oracle/ (a dropped term, a sign, a
transposed operand, a wrong index) makes one of these fail."""
import json
import math
import os

import numpy as np
import pytest

import synth
from oracle import core, dense, rng


def tiny_problem(m, n, nnz, seed=3, lam=0.1, rank=2):
    return synth.tiny(m, n, nnz, rank=rank, lam=lam, seed=seed)


def rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


# ----------------------------------------------------------------------------- RNG

def test_splitmix64_reference_values(golden_dir):
    """The counter generator reproduces the published SplitMix64 outputs."""
    vals = [int(l) for l in open(os.path.join(golden_dir, "splitmix64_seed1234567.txt"))
            if l.strip() and not l.startswith("#")]
    got = [int(v) for v in rng.raw_draws(1234567, 0, 5)]
    assert got == vals


def test_normals_moments_and_streams():
    z = rng.normals(5, 1, 200_000)
    assert abs(z.mean()) < 0.01 and abs(z.var() - 1.0) < 0.01
    assert abs(np.mean(z ** 4) - 3.0) < 0.05
    z2 = rng.normals(5, 2, 1000)
    assert not np.allclose(z[:1000], z2)
    # prefix property: entry i does not depend on the count drawn
    assert np.array_equal(rng.normals(9, 3, 10), rng.normals(9, 3, 50)[:10])


# ----------------------------------------------------------------------------- sparse loops

@pytest.mark.parametrize("m,n,nnz", [(7, 11, 30), (11, 7, 40), (5, 9, 45), (9, 5, 1), (6, 6, 0),
                                     (30, 17, 200)])
def test_sparse_products_match_masked_dense(m, n, nnz):
    p = tiny_problem(m, n, nnz)
    A, M = dense.to_dense(p)
    for k in (1, 3, 8):
        W, H = rand((m, k), 1), rand((n, k), 2)
        R = core.sddmm(p, W, H)
        Rd = np.where(M, W @ H.T - A, 0.0)
        assert np.allclose(R, Rd[M], rtol=0, atol=1e-13)
        assert np.allclose(core.sddmm(p, W, H, with_values=False), (W @ H.T)[M], atol=1e-13)
        S = rand(p.nnz, 4)
        Sd = np.zeros((m, n))
        Sd[M] = S
        B, U = rand((n, 5), 5), rand((m, 6), 6)
        assert np.allclose(core.spmm(p, S, B), Sd @ B, atol=1e-12)
        assert np.allclose(core.spmm_t(p, S, U), Sd.T @ U, atol=1e-12)
        assert math.isclose(core.sumsq(p, R), float(np.sum(Rd ** 2)), rel_tol=1e-13, abs_tol=1e-300)


def test_row_order_of_omega_matches_dense_mask():
    # CSR order is row-major: boolean-mask indexing of the dense matrix has the same order
    p = tiny_problem(9, 13, 50)
    A, M = dense.to_dense(p)
    assert np.array_equal(A[M], p.val)


# ----------------------------------------------------------------------------- objectives

def test_nuclear_norm_factored_vs_dense():
    for k in (1, 3, 6):
        W, H = rand((20, k), k), rand((15, k), k + 10)
        assert math.isclose(core.nuclear_norm(W, H),
                            np.linalg.svd(W @ H.T, compute_uv=False).sum(), rel_tol=1e-12)


def test_balanced_factors_attain_nuclear_norm():
    """Lemma 'equivalent': ||X||_* = min 1/2(||W||^2 + ||H||^2), attained at W = U sqrt(S)."""
    X = rand((12, 4), 1) @ rand((4, 18), 2)
    U, s, Vt = np.linalg.svd(X, full_matrices=False)
    W, H = U[:, :4] * np.sqrt(s[:4]), Vt[:4].T * np.sqrt(s[:4])
    assert math.isclose(0.5 * (np.sum(W ** 2) + np.sum(H ** 2)), s.sum(), rel_tol=1e-12)
    Q = np.linalg.qr(rand((4, 4), 3))[0] * 1.7   # any other factorisation is not smaller
    W2, H2 = W @ Q, H @ np.linalg.inv(Q).T
    assert np.allclose(W2 @ H2.T, X)
    assert 0.5 * (np.sum(W2 ** 2) + np.sum(H2 ** 2)) > s.sum()


def test_eq_trace_identity_with_corrected_sign():
    W1, H1, W0, H0 = rand((10, 3), 1), rand((14, 3), 2), rand((10, 2), 3), rand((14, 2), 4)
    d = np.sum((W1 @ H1.T - W0 @ H0.T) ** 2)
    assert math.isclose(core.diff_fro2_factored(W1, H1, W0, H0), d, rel_tol=1e-12)


def test_step_norm_split_matches_dense():
    Wt, Ht = rand((12, 3), 1), rand((16, 3), 2)
    Uhat = np.linalg.qr(rand((12, 5), 3))[0]
    Wn, Hn = Uhat @ rand((5, 2), 4), rand((16, 2), 5)   # ran(Wn) inside ran(Uhat)
    d = np.linalg.norm(Wt @ Ht.T - Wn @ Hn.T)
    assert math.isclose(core.step_norm(Uhat, Wt, Ht, Wn, Hn), d, rel_tol=1e-12)


# ----------------------------------------------------------------------------- BM phase

def test_bm_half_step_is_exact_line_search_and_monotone():
    p = tiny_problem(30, 40, 500, lam=0.3)
    W, H = rand((30, 4), 1), rand((40, 4), 2)
    lam = 0.3
    R = core.sddmm(p, W, H)
    G = core.spmm(p, R, H) + lam * W
    D = -G @ np.linalg.inv(H.T @ H + lam * np.eye(4))
    W1, s = core.bm_half_step_W(p, W, H, lam)
    assert s > 0 and np.allclose(W1, W + s * D)
    phi = lambda t: core.bm_objective(p, W + t * D, H, lam)   # noqa: E731
    # the quadratic's minimiser: neighbours on both sides are not lower
    for d in (1e-3, 1e-2):
        assert phi(s) <= phi(s * (1 + d)) and phi(s) <= phi(s * (1 - d))
    # brute-force minimiser of the 1-D quadratic from three samples
    f0, f1, f2 = phi(0.0), phi(s), phi(2 * s)
    a = (f2 - 2 * f1 + f0) / (2 * s * s)
    b = (f1 - f0) / s - a * s
    assert math.isclose(-b / (2 * a), s, rel_tol=1e-6)
    # non-increase over epochs (eq. nonincrease)
    Fs = [core.bm_objective(p, W, H, lam)]
    for _ in range(5):
        W, H, _ = core.bm_epoch(p, W, H, lam)
        Fs.append(core.bm_objective(p, W, H, lam))
    assert all(b <= a + 1e-12 * abs(a) for a, b in zip(Fs, Fs[1:]))


def test_bm_H_step_matches_transposed_W_step():
    p = tiny_problem(25, 35, 300)
    pt = core.transpose(p)
    assert np.array_equal(pt.col, _transpose(p)[1]) and np.array_equal(pt.val, _transpose(p)[2])
    W, H = rand((25, 3), 1), rand((35, 3), 2)
    H1, s1 = core.bm_half_step_H(p, W, H, 0.2)
    H2, s2 = core.bm_half_step_W(pt, H, W, 0.2)
    assert math.isclose(s1, s2, rel_tol=1e-12) and np.allclose(H1, H2, atol=1e-12)


def _transpose(p):
    rows = p.rows()
    order = np.lexsort((rows, p.col))
    col_t = rows[order].astype(np.int32)
    rp = np.zeros(p.n + 1, np.int64)
    np.cumsum(np.bincount(p.col, minlength=p.n), out=rp[1:])
    return rp, col_t, p.val[order]


# ----------------------------------------------------------------------------- orth / LmSVD / prox

def test_orth_spans_and_cuts_rank():
    a, b = rand((50, 3), 1), rand((50, 2), 2)
    M = np.column_stack([a, b, a @ rand((3, 2), 3), 1e-9 * rand((50, 1), 4) + b[:, :1]])
    Q = core.orth(M)
    assert Q.shape[1] == 5
    assert np.allclose(Q.T @ Q, np.eye(5), atol=1e-12)
    P = Q @ Q.T
    assert np.allclose(P @ a, a, atol=1e-10) and np.allclose(P @ b, b, atol=1e-10)
    assert core.orth(np.zeros((5, 3))).shape[1] == 0


def _dense_Z(p, W, H, alpha):
    A, M = dense.to_dense(p)
    X = W @ H.T
    return X - alpha * np.where(M, X - A, 0.0)


def test_lmsvd_finds_dominant_subspace():
    p = tiny_problem(40, 60, 900, lam=0.2)
    W, H = rand((40, 3), 1), rand((60, 3), 2)
    alpha = 1.99
    z = core.ZOperator(p, W, H, core.sddmm(p, W, H), alpha)
    Z = _dense_Z(p, W, H, alpha)
    assert np.allclose(z.matmul(rand((60, 2), 5)), Z @ rand((60, 2), 5), atol=1e-10)
    assert np.allclose(z.rmatmul(rand((40, 2), 6)), Z.T @ rand((40, 2), 6), atol=1e-10)
    assert math.isclose(z.fro2(), float(np.sum(Z * Z)), rel_tol=1e-10)
    U0 = core.orth(rand((40, 6), 7))
    ls = core.lmsvd(z, U0, 1e-14, max_iter=500)
    ev = np.sort(np.linalg.eigvalsh(Z @ Z.T))[::-1]
    assert np.allclose(ls.ritz[:3], ev[:3], rtol=1e-10)
    s = np.linalg.svd(Z, compute_uv=False)
    assert np.allclose(np.linalg.svd(ls.Y, compute_uv=False)[:3], s[:3], rtol=1e-9)


class _DenseOp:
    """Z given as a dense matrix, with the two products Algorithm 2 uses."""

    def __init__(self, Z):
        self.Z = Z

    def matmul(self, B):
        return self.Z @ B

    def rmatmul(self, U):
        return self.Z.T @ U


def _slow_spectrum(m, n, decay, seed):
    """Z = U diag(decay^j) V^T with random orthonormal U, V: eigenvalues of Z Z^T
    so close that the block subspace iteration converges slowly."""
    r = min(m, n)
    Uz = np.linalg.qr(rand((m, r), seed))[0]
    Vz = np.linalg.qr(rand((n, r), seed + 1))[0]
    s = decay ** np.arange(r)
    return Uz @ np.diag(s) @ Vz.T, s


@pytest.mark.parametrize("p", [1, 2])
def test_lmsvd_history_ritz_values_are_optimal_over_the_subspace(p):
    # eqs. PUi, orth-W, lmsvd-opt: the k_t Ritz values are the leading eigenvalues
    # of Z Z^T compressed onto ran(U^{t,i}, ..., U^{t,i-p}), whose basis here comes
    # from an SVD of the stacked blocks (not from the projection of eq. PUi)
    Z, _ = _slow_spectrum(60, 90, 0.98, 11)
    kt = 4
    tr = []
    core.lmsvd(_DenseOp(Z), rand((60, kt), 12), 0.0, max_iter=6, p=p, trace=tr)
    assert len(tr) == 6
    checked = 0
    for i, rec in enumerate(tr):
        Q, Uold = rec["Q"], rec["Uold"]
        assert np.allclose(Q.T @ Q, np.eye(Q.shape[1]), atol=1e-12)
        if i == 0:
            assert Uold is None and Q.shape[1] == kt
            continue
        assert Uold.shape[1] == kt * min(p, i)
        # the inputs keep every history direction well away from the cut
        assert rec["lam"].min() > 10 * core.LMSVD_EIG_TOL
        Ui = Q[:, :kt]
        Ub, sb, _ = np.linalg.svd(np.column_stack([Ui, Uold]), full_matrices=False)
        B = Ub[:, sb > 1e-8]
        assert B.shape[1] == Q.shape[1]
        assert np.allclose(B @ (B.T @ Q), Q, atol=1e-10)
        ev = np.sort(np.linalg.eigvalsh(B.T @ Z @ Z.T @ B))[::-1][:kt]
        assert np.allclose(rec["theta"], ev, rtol=1e-11, atol=1e-14)
        checked += 1
    assert checked == 5


def test_lmsvd_history_reaches_dominant_subspace_in_fewer_iterations():
    # Algorithm 2 with p >= 1 converges to the same leading eigenpairs as p = 0
    # (dense eigendecomposition) and, on a slowly decaying spectrum, in fewer
    # iterations: the point of the history blocks
    Z, s = _slow_spectrum(80, 120, 0.95, 21)
    kt = 5
    U0 = rand((80, kt), 22)
    its = {}
    for p in (0, 1, 2):
        ls = core.lmsvd(_DenseOp(Z), U0, 1e-13, max_iter=2000, p=p)
        its[p] = ls.iters
        assert ls.iters < 2000
        assert np.allclose(ls.ritz, s[:kt] ** 2, rtol=1e-9)
        Pu = ls.Uhat @ ls.Uhat.T
        Ud = np.linalg.svd(Z)[0][:, :kt]
        assert np.allclose(Pu @ Ud, Ud, atol=1e-5)
    assert its[1] < 0.8 * its[0] and its[2] < its[1]


def test_solve_with_lmsvd_history_matches_dense_proximal_gradient():
    p = tiny_problem(40, 60, 700, lam=0.3, rank=3, seed=5)
    A, M = dense.to_dense(p)
    Xd, _ = dense.proximal_gradient_dense(A, M, 0.3, alpha=1.99, tol=1e-14)
    Fd = dense.mc_objective_dense(Xd, A, M, 0.3)
    for hp in (1, 2):
        res = core.solve(p, core.Options(lam=0.3, k0=4, tol=1e-11, seed=3, lmsvd_p=hp))
        assert res.converged
        assert math.isclose(res.F, Fd, rel_tol=1e-11)
        assert np.allclose((res.W @ res.H.T)[M], Xd[M], atol=1e-6)


def test_prox_with_full_basis_equals_closed_form():
    """eq. proxnuc: with Uhat spanning R^m the inexact step is the exact prox."""
    p = tiny_problem(12, 20, 120, lam=0.4)
    W, H = rand((12, 3), 1), rand((20, 3), 2)
    alpha, lam = 1.99, 0.4
    z = core.ZOperator(p, W, H, core.sddmm(p, W, H), alpha)
    Uhat = np.eye(12)
    pr = core.prox_from_basis(Uhat, z.rmatmul(Uhat), alpha * lam)
    Xp = dense.prox_nuclear(_dense_Z(p, W, H, alpha), alpha * lam)
    assert np.allclose(pr.W @ pr.H.T, Xp, atol=1e-11)
    assert pr.k == np.linalg.matrix_rank(Xp, tol=1e-9)
    # balanced output: 1/2(||W||^2 + ||H||^2) = sum of the kept singular values
    assert math.isclose(0.5 * (np.sum(pr.W ** 2) + np.sum(pr.H ** 2)), pr.sigma.sum(), rel_tol=1e-12)


def test_inexact_prox_error_bound():
    """prox is 1-Lipschitz, so ||X+ - prox(Z)|| <= ||Z~ - Z|| (the eq. C5-1 bound)."""
    p = tiny_problem(30, 45, 600, lam=0.3)
    W, H = rand((30, 2), 1), rand((45, 2), 2)
    alpha, lam = 1.99, 0.3
    Z = _dense_Z(p, W, H, alpha)
    pr, ls, _ = core.prox_step_standalone(p, W, H, lam, alpha, seed=4, tau=1e-6, max_iter=3)
    Zt = ls.Uhat @ (ls.Uhat.T @ Z)
    Xp = dense.prox_nuclear(Z, alpha * lam)
    assert np.linalg.norm(pr.W @ pr.H.T - Xp) <= np.linalg.norm(Zt - Z) * (1 + 1e-9) + 1e-12


def test_safeguard_column_properties():
    U = np.linalg.qr(rand((30, 4), 1))[0]
    u = rand(30, 2)
    c = core.safeguard_column(U, u, 0.1, seed=3, t=2)
    ut = u - U @ (U.T @ u)
    xi = c - ut
    assert np.allclose(U.T @ c, 0, atol=1e-12)
    assert math.isclose(np.linalg.norm(xi), 0.1, rel_tol=1e-12)
    assert abs(xi @ ut) < 1e-12
    c0 = core.safeguard_column(U, None, 0.1, seed=3, t=2)
    assert math.isclose(np.linalg.norm(c0), 1.0, rel_tol=1e-12) and np.allclose(U.T @ c0, 0, atol=1e-12)


def test_initialize_is_exact_prox_when_sketch_covers_range():
    """With k0 >= m the range finder captures ran(P_Omega(A)); the first step is
    then exactly SVT_lambda(P_Omega(A)) (alpha_{-1} = 1, X_{-1} = 0)."""
    p = tiny_problem(10, 25, 100, lam=0.5)
    A, M = dense.to_dense(p)
    init, _ = core.initialize(p, 0.5, 12, seed=1)
    assert np.allclose(init.W @ init.H.T, dense.prox_nuclear(A, 0.5), atol=1e-10)


# ----------------------------------------------------------------------------- end to end

def test_full_omega_closed_form():
    """Omega = all entries: X* = SVT_lambda(A) (soft-impute fixed point)."""
    m, n, lam = 15, 22, 1.0
    p = tiny_problem(m, n, m * n, lam=lam, rank=3)
    A, _ = dense.to_dense(p)
    res = core.solve(p, core.Options(lam=lam, k0=4, tol=1e-12, seed=2))
    Xs = dense.prox_nuclear(A, lam)
    assert res.converged
    assert np.allclose(res.W @ res.H.T, Xs, atol=1e-9)
    F_star = dense.mc_objective_dense(Xs, A, np.ones_like(A, bool), lam)
    assert math.isclose(res.F, F_star, rel_tol=1e-12)


def test_solve_tall_problem_equals_transposed_solve():
    p = tiny_problem(45, 30, 500, lam=0.3, rank=2, seed=10)
    a = core.solve(p, core.Options(lam=0.3, k0=4, tol=1e-11, seed=3))
    A, M = dense.to_dense(p)
    Xd, _ = dense.proximal_gradient_dense(A, M, 0.3, alpha=1.99, tol=1e-14)
    assert a.W.shape[0] == 45 and a.H.shape[0] == 30
    assert math.isclose(a.F, dense.mc_objective_dense(Xd, A, M, 0.3), rel_tol=1e-11)


def test_solve_matches_dense_proximal_gradient():
    p = tiny_problem(40, 60, 700, lam=0.3, rank=3, seed=5)
    A, M = dense.to_dense(p)
    res = core.solve(p, core.Options(lam=0.3, k0=4, tol=1e-11, seed=3))
    Xd, _ = dense.proximal_gradient_dense(A, M, 0.3, alpha=1.99, tol=1e-14)
    Fd = dense.mc_objective_dense(Xd, A, M, 0.3)
    assert res.converged
    assert math.isclose(res.F, Fd, rel_tol=1e-11)
    assert res.k == np.linalg.matrix_rank(Xd, tol=1e-7)
    # X* itself is unique here only on Omega up to the solution set; compare there
    assert np.allclose((res.W @ res.H.T)[M], Xd[M], atol=1e-6)


def test_solve_optimality_conditions_and_monotone_bm():
    p = tiny_problem(50, 70, 1200, lam=0.25, rank=3, seed=8)
    recs = []
    res = core.solve(p, core.Options(lam=0.25, k0=5, tol=1e-11, seed=4), callback=recs.append)
    assert res.converged
    X = res.W @ res.H.T
    A, M = dense.to_dense(p)
    G = np.where(M, X - A, 0.0)
    U, s, Vt = np.linalg.svd(X)
    k = res.k
    U, V = U[:, :k], Vt[:k].T
    # -G in lambda * subdifferential of the nuclear norm at X
    assert np.allclose(G @ V, -0.25 * U, atol=1e-7)
    assert np.allclose(G.T @ U, -0.25 * V, atol=1e-7)
    assert np.linalg.svd(G, compute_uv=False)[0] <= 0.25 * (1 + 1e-7)
    # F of the balanced prox output is never below F~ at the same point; F~ after BM <= F before it
    Fs = [r.F for r in recs]
    assert all(r.F_bm <= f_prev * (1 + 1e-12) for r, f_prev in zip(recs[1:], Fs))


def test_duality_gap_certifies_oracle():
    p = tiny_problem(60, 80, 1500, lam=0.4, rank=3, seed=9)
    res = core.solve(p, core.Options(lam=0.4, k0=4, tol=1e-11, seed=5))
    _, R = core.loss(p, res.W, res.H)
    gap, D, g2 = dense.duality_gap(p, R, res.F, 0.4)
    assert gap >= -1e-9 * res.F
    assert gap <= 1e-8 * res.F


def test_large_lambda_gives_zero_solution():
    """lambda >= ||P_Omega(A)||_2: X* = 0 (rank 0) and F* = 1/2 ||A_Omega||^2."""
    p = tiny_problem(20, 30, 200, seed=6)
    A, _ = dense.to_dense(p)
    lam = 1.01 * np.linalg.svd(A, compute_uv=False)[0]
    res = core.solve(p, core.Options(lam=lam, k0=4, tol=1e-10, seed=1))
    assert res.k == 0
    assert math.isclose(res.F, 0.5 * float(np.sum(p.val ** 2)), rel_tol=1e-14)


def test_empty_omega():
    p = tiny_problem(8, 9, 0)
    res = core.solve(p, core.Options(lam=0.1, k0=3, tol=1e-10, seed=1))
    assert res.k == 0 and res.F == 0.0


def test_golden_small_uniform_is_certified(golden_dir):
    """The stored oracle optimum of the 1000 x 1500 workload carries a duality
    gap certificate: F* is within that gap of the true minimum."""
    g = json.load(open(os.path.join(golden_dir, "small_uniform.json")))
    assert g["converged"] and g["residual"] <= 1e-10
    assert 0 <= g["dual_gap"] <= 1e-8 * g["F"]
    assert g["dual_value"] <= g["F"]


# ----------------------------------------------------------------------------- SpaRSA step

def test_bb_step_matches_dense_definition():
    # eq. proxBB read as ||dX||^2 / <dX, d grad f>, with grad f = P_Omega(X - A)
    p = tiny_problem(30, 45, 500, lam=0.2)
    A, M = dense.to_dense(p)
    W, H, Wp, Hp = rand((30, 3), 1), rand((45, 3), 2), rand((30, 2), 3), rand((45, 2), 4)
    R, Rp = core.sddmm(p, W, H), core.sddmm(p, Wp, Hp)
    dX = W @ H.T - Wp @ Hp.T
    dG = np.where(M, W @ H.T - A, 0.0) - np.where(M, Wp @ Hp.T - A, 0.0)
    want = float(np.sum(dX * dX)) / float(np.sum(dX * dG))
    assert 1.0 < want < 1e3
    assert math.isclose(core.bb_step(W, H, Wp, Hp, R, Rp, 1e-3, 1e6), want, rel_tol=1e-10)
    assert core.bb_step(W, H, Wp, Hp, R, Rp, 2 * want, 1e6) == 2 * want
    assert core.bb_step(W, H, Wp, Hp, R, Rp, 1e-3, 0.5 * want) == 0.5 * want
    assert core.bb_step(W, H, W, H, R, R, 1.0, 7.0) == 7.0


def test_diff_fro2_split_resolves_nearby_iterates():
    W1, H1, V = rand((40, 4), 1), rand((60, 4), 2), rand((40, 4), 3)
    W0, H0 = rand((40, 3), 4), rand((60, 3), 5)
    d = float(np.sum((W1 @ H1.T - W0 @ H0.T) ** 2))
    assert math.isclose(core.diff_fro2_split(W1, H1, W0, H0), d, rel_tol=1e-12)
    # W0 = W1 + delta V, H0 = H1: dX = -delta V H1^T exactly
    for delta in (1e-4, 1e-9, 1e-12):
        exact = delta ** 2 * float(np.sum((V @ H1.T) ** 2))
        got = core.diff_fro2_split(W1, H1, W1 + delta * V, H1)
        assert math.isclose(got, exact, rel_tol=1e-3), (delta, got, exact)
    # where eq. trace has lost every digit
    three = core.diff_fro2_factored(W1, H1, W1 + 1e-9 * V, H1)
    assert not math.isclose(three, 1e-18 * float(np.sum((V @ H1.T) ** 2)), rel_tol=1e-1)


def test_back_condition_matches_dense_definition():
    p = tiny_problem(30, 45, 500, lam=0.2)
    A, M = dense.to_dense(p)
    W, H, Wn, Hn = rand((30, 3), 5), rand((45, 3), 6), rand((30, 2), 7), rand((45, 2), 8)
    X, Xn = W @ H.T, Wn @ Hn.T
    f = lambda Y: 0.5 * float(np.sum(np.where(M, Y - A, 0.0) ** 2))  # noqa: E731
    G = np.where(M, X - A, 0.0)
    d2 = float(np.sum((Xn - X) ** 2))
    for alpha, delta in [(1.99, 0.999), (50.0, 0.5), (0.1, 0.9), (2.1, 0.9)]:
        rhs = f(X) + float(np.sum(G * (Xn - X))) + delta / alpha * d2
        ok, lhs, r = core.back_condition(p, core.sddmm(p, W, H), Wn, Hn, d2, alpha, delta)
        # the curvature term of the quadratic loss, and the literal eq. back
        assert math.isclose(lhs, f(Xn) - f(X) - float(np.sum(G * (Xn - X))), rel_tol=1e-9)
        assert math.isclose(r, delta / alpha * d2, rel_tol=1e-12)
        assert ok == (f(Xn) <= rhs)
    assert not core.back_condition(p, core.sddmm(p, W, H), Wn, Hn, d2, 50.0, 0.5)[0]
    # any step alpha < 2 delta / L (L = 1) satisfies it: the descent lemma
    ok, _, _ = core.back_condition(p, core.sddmm(p, W, H), Wn, Hn, d2, 1.99, 0.999)
    assert ok


def test_sparsa_with_equal_bounds_is_the_fixed_step():
    p = tiny_problem(40, 60, 700, lam=0.3, rank=3, seed=5)
    ra, rb = [], []
    a = core.solve(p, core.Options(lam=0.3, k0=4, tol=1e-9, seed=3), callback=ra.append)
    b = core.solve(p, core.Options(lam=0.3, k0=4, tol=1e-9, seed=3, step_rule="sparsa",
                                   alpha_min=1.99, alpha_max=1.99), callback=rb.append)
    assert a.iters == b.iters and np.array_equal(a.W, b.W) and np.array_equal(a.H, b.H)
    assert [r.residual for r in ra] == [r.residual for r in rb]
    assert all(r.trials == 1 and r.alpha == 1.99 for r in rb)


def test_sparsa_solve_reaches_the_optimum_in_fewer_iterations():
    # the SpaRSA variant: same optimum as the dense proximal gradient, fewer outer
    # iterations than the fixed step, paid for with backtracking prox computations
    p = synth.tiny(300, 500, 30000, rank=8, lam=1.0, seed=4)
    fx, sp = [], []
    a = core.solve(p, core.Options(lam=1.0, k0=8, tol=1e-9, seed=1), callback=fx.append)
    b = core.solve(p, core.Options(lam=1.0, k0=8, tol=1e-9, seed=1, step_rule="sparsa"),
                   callback=sp.append)
    assert a.converged and b.converged
    # optimality of the SpaRSA output certified by the dual (no solver involved)
    _, R = core.loss(p, b.W, b.H)
    gap, _, _ = dense.duality_gap(p, R, b.F, 1.0)
    assert -1e-9 * b.F <= gap <= 5e-8 * b.F      # the fixed step at this tol: 1.0e-8
    assert math.isclose(b.F, a.F, rel_tol=1e-10)
    assert b.iters < a.iters
    assert sum(r.trials for r in sp) > b.iters
    assert all(1.99 <= r.alpha <= 1e3 for r in sp) and max(r.alpha for r in sp) > 1.99


# ----------------------------------------------------------------------------- polyMF-SS

def test_polymf_block_direction_and_exact_quartic_step():
    # Sec. 6.1.1: a block is column j of W and of H; exact line search
    p = tiny_problem(30, 45, 600, lam=0.3)
    A, M = dense.to_dense(p)
    lam, j = 0.3, 1
    W, H = rand((30, 3), 11), rand((45, 3), 12)
    R = core.sddmm(p, W, H)
    W1, H1, R1, t = core.polymf_block(p, W, H, j, lam, R)
    G = np.where(M, W @ H.T - A, 0.0)
    w, h = W[:, j], H[:, j]
    dw = -(G @ h + lam * w) / (M @ (h * h) + lam)
    dh = -(G.T @ w + lam * h) / (M.T @ (w * w) + lam)
    assert t > 0
    assert np.allclose(W1[:, j], w + t * dw, atol=1e-12) and np.allclose(H1[:, j], h + t * dh, atol=1e-12)
    assert np.array_equal(np.delete(W1, j, 1), np.delete(W, j, 1))
    # the updated residual is the residual of the new factors
    assert np.allclose(R1, core.sddmm(p, W1, H1), atol=1e-12)

    def phi(s):
        Ws, Hs = W.copy(), H.copy()
        Ws[:, j] = w + s * dw
        Hs[:, j] = h + s * dh
        return 0.5 * float(np.sum(np.where(M, Ws @ Hs.T - A, 0.0) ** 2)) \
            + 0.5 * lam * (float(np.sum(Ws * Ws)) + float(np.sum(Hs * Hs)))
    grid = np.linspace(0.0, 3.0 * t + 1.0, 3001)
    vals = np.array([phi(s) for s in grid])
    assert phi(t) <= vals.min() + 1e-12 * abs(vals.min())
    e = 1e-5 * t
    assert abs(phi(t + e) - phi(t - e)) / (2 * e) <= 1e-6 * abs(phi(0.0) - phi(t)) / t


def test_quartic_min_cases():
    # psi(t) = c1 t + c2 t^2 + c3 t^3 + c4 t^4 over t >= 0
    assert core.quartic_min(-2.0, 1.0, 0.0, 0.0) == pytest.approx(1.0)       # quadratic
    assert core.quartic_min(1.0, 1.0, 0.0, 0.0) == 0.0                        # ascent
    # two local minima (roots of psi' at 1, 2, 4 scaled): the global one wins
    # psi'(t) = 4 (t - 1)(t - 2)(t - 4) = 4 t^3 - 28 t^2 + 56 t - 32
    c4, c3, c2, c1 = 1.0, -28.0 / 3, 28.0, -32.0
    psi = lambda s: ((c4 * s + c3) * s + c2) * s * s + c1 * s  # noqa: E731
    best = min((1.0, 4.0), key=psi)
    assert best == 4.0 and core.quartic_min(c1, c2, c3, c4) == pytest.approx(best, rel=1e-9)
    # psi'(t) = 4 (t - 1)(t - 3)(t - 4): here the nearer minimum t = 1 is the global one
    c4, c3, c2, c1 = 1.0, -32.0 / 3, 38.0, -48.0
    assert core.quartic_min(c1, c2, c3, c4) == pytest.approx(1.0, rel=1e-9)


def test_polymf_epoch_is_monotone_and_solves():
    p = tiny_problem(40, 60, 700, lam=0.3, rank=3, seed=5)
    A, M = dense.to_dense(p)
    W, H = rand((40, 4), 1), rand((60, 4), 2)
    F = [core.bm_objective(p, W, H, 0.3)]
    for _ in range(4):
        R = core.sddmm(p, W, H)
        for j in range(4):
            W, H, R, _ = core.polymf_block(p, W, H, j, 0.3, R)
            F.append(core.bm_objective(p, W, H, 0.3))
    assert all(b <= a * (1 + 1e-14) for a, b in zip(F, F[1:])) and F[-1] < F[0]
    res = core.solve(p, core.Options(lam=0.3, k0=4, tol=1e-11, seed=3, bm_solver="polymf"))
    Xd, _ = dense.proximal_gradient_dense(A, M, 0.3, alpha=1.99, tol=1e-14)
    assert res.converged
    assert math.isclose(res.F, dense.mc_objective_dense(Xd, A, M, 0.3), rel_tol=1e-11)
