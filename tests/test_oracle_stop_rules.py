"""Pins of the oracle's stop rules: the normalised optimality residuals that end
every solve and define every time-to-tolerance figure (CPU only).

The paper leaves the matrix-completion residual undefined (Sec. 6.1 calls the
exact prox-gradient norm impractical); the reading taken is
    res(X~) = ||X~ - prox_{alpha lam ||.||_*}(X~ - alpha grad f(X~))||_F
              / (1 + ||X~||_F + ||grad f(X~)||_F),        grad f = P_Omega(X~ - A).
For the kernel-estimation QSDP (Sec. 6.2) the stop residual is the
prox-gradient mapping ||X~ - X+||_F / alpha over (1 + ||X~||_F + ||grad f~||_F)
with grad f~ = A^*(A(X~) - b) + lam I.

Each pin computes the value from explicit dense matrices by a route the
oracle does not take (full SVDs, a finite-difference gradient of the dense
objective, the projection in reduced coordinates), and each pin is shown to
reject the plausible slips in the normalisation (a dropped "1 +", squared
norms, a doubled off-diagonal, a missing or extra step-size factor)."""
import math

import numpy as np
import pytest

import synth
from oracle import core, rke


def rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


# ----------------------------------------------------------------------------- matrix completion

def mc_dense_residual(p, W, H, lam, alpha):
    """The reading's residual from explicit matrices: full SVD of the PG point."""
    A = np.zeros((p.m, p.n))
    M = np.zeros((p.m, p.n), bool)
    A[p.rows(), p.col] = p.val
    M[p.rows(), p.col] = True
    X = W @ H.T
    G = np.where(M, X - A, 0.0)
    U, s, Vt = np.linalg.svd(X - alpha * G, full_matrices=False)
    Xp = (U * np.maximum(s - alpha * lam, 0.0)) @ Vt
    return np.linalg.norm(X - Xp) / (1.0 + np.linalg.norm(X) + np.linalg.norm(G))


# (m, n, nnz, k, lam, alpha): k + 1 >= min(m, n), so the warm-started basis of the
# oracle's PG step spans the whole short side and its prox is the exact one
MC_CASES = [(6, 11, 40, 5, 0.3, 1.99), (6, 11, 40, 5, 0.3, 1.0), (7, 9, 63, 6, 0.05, 1.99),
            (10, 6, 45, 5, 0.4, 1.99), (5, 14, 30, 4, 2.0, 1.99)]


def _mc_parts(case, scale):
    m, n, nnz, k, lam, alpha = case
    p = synth.tiny(m, n, nnz, rank=2, lam=lam, seed=m + n + k)
    W, H = scale * rand((m, k), 1), scale * rand((n, k), 2)
    pr, ls, res = core.prox_step_standalone(p, W, H, lam, alpha, seed=3, tau=1e-15, max_iter=400)
    return p, W, H, lam, alpha, pr, ls, res


def mc_pin_holds(residual_fn, rtol=1e-9):
    """True when residual_fn(p, W~, H~, R, Uhat, W+, H+, alpha) equals the dense
    residual on every case (two factor scales: norms below and above 1)."""
    for case in MC_CASES:
        for scale in (0.3, 1.7):
            p, W, H, lam, alpha, pr, ls, _ = _mc_parts(case, scale)
            if p.m > p.n:   # the oracle works on the transpose; so does the pin
                pt = core.transpose(p)
                got = residual_fn(pt, H, W, core.sddmm(pt, H, W), ls.Uhat, pr.H, pr.W, alpha)
            else:
                got = residual_fn(p, W, H, core.sddmm(p, W, H), ls.Uhat, pr.W, pr.H, alpha)
            if not math.isclose(got, mc_dense_residual(p, W, H, lam, alpha), rel_tol=rtol):
                return False
    return True


def test_mc_relative_residual_matches_dense_definition():
    """relative_residual (used by every solve and PG step of the oracle) equals
    the reading's residual computed from full SVDs; so does the value the
    oracle's standalone PG step reports, also for m > n."""
    assert mc_pin_holds(lambda p, W, H, R, U, Wn, Hn, a: core.relative_residual(p, W, H, R, U, Wn, Hn))
    for case in MC_CASES:
        p, W, H, lam, alpha, _, _, res = _mc_parts(case, 0.8)
        assert math.isclose(res, mc_dense_residual(p, W, H, lam, alpha), rel_tol=1e-9)


def test_mc_residual_at_the_optimum_and_far_from_it():
    """At the dense optimum the residual vanishes; at X~ = 0 with lambda below
    ||P_Omega(A)||_2 it is ||prox(alpha A_Omega)|| / (1 + ||A_Omega||)."""
    p = synth.tiny(8, 12, 60, rank=2, lam=0.2, seed=21)
    A = np.zeros((8, 12)); M = np.zeros((8, 12), bool)
    A[p.rows(), p.col] = p.val; M[p.rows(), p.col] = True
    X = np.zeros((8, 12))
    for _ in range(20000):   # soft-impute to its fixed point
        U, s, Vt = np.linalg.svd(X - np.where(M, X - A, 0.0), full_matrices=False)
        Xn = (U * np.maximum(s - 0.2, 0.0)) @ Vt
        if np.linalg.norm(Xn - X) < 1e-15 * (1 + np.linalg.norm(X)):
            break
        X = Xn
    U, s, Vt = np.linalg.svd(X, full_matrices=False)
    r = int(np.sum(s > 1e-10))
    W, H = U[:, :r] * np.sqrt(s[:r]), Vt[:r].T * np.sqrt(s[:r])
    Wp = np.zeros((8, 7)); Hp = np.zeros((12, 7))
    Wp[:, :r], Hp[:, :r] = W, H
    _, _, res = core.prox_step_standalone(p, Wp, Hp, 0.2, 1.99, seed=1, tau=1e-15, max_iter=400)
    assert res < 1e-12
    # X~ = W H^T ~ 1e-28 (factors of full width so the basis spans R^m): the
    # closed form at X~ = 0, alpha = 1
    W0, H0 = 1e-14 * rand((8, 7), 4), 1e-14 * rand((12, 7), 5)
    _, _, res0 = core.prox_step_standalone(p, W0, H0, 0.2, 1.0, seed=1, tau=1e-15, max_iter=400)
    s0 = np.linalg.svd(A, compute_uv=False)
    expect = np.sqrt(np.sum(np.maximum(s0 - 0.2, 0.0) ** 2)) / (1.0 + np.linalg.norm(p.val))
    assert math.isclose(res0, expect, rel_tol=1e-10)


def _mc_slip(kind):
    def fn(p, W, H, R, U, Wn, Hn, alpha):
        d = core.step_norm(U, W, H, Wn, Hn)
        x = math.sqrt(core.fro2_factored(W, H))
        g = math.sqrt(core.sumsq(p, R))
        if kind == "no_one":
            return d / (x + g)
        if kind == "squared_norms":
            return d / (1.0 + x * x + g * g)
        if kind == "squared_step":
            return d * d / (1.0 + x + g)
        if kind == "values_not_gradient":
            return d / (1.0 + x + math.sqrt(float(np.dot(p.val, p.val))))
        if kind == "divided_by_alpha":
            return d / (alpha * (1.0 + x + g))
        raise ValueError(kind)
    return fn


@pytest.mark.parametrize("kind", ["no_one", "squared_norms", "squared_step", "values_not_gradient",
                                  "divided_by_alpha"])
def test_mc_residual_pin_rejects_planted_slips(kind):
    assert not mc_pin_holds(_mc_slip(kind))


# ----------------------------------------------------------------------------- kernel-estimation QSDP

def qsdp_dense_f(p, X, lam):
    """f(X) + lam tr(X), f = 1/2 sum over pairs (X_ii + X_jj - 2 X_ij - d_ij^2)^2
    (stored entries count every pair twice)."""
    rows, cols = p.rows(), p.col
    r = X[rows, rows] + X[cols, cols] - 2.0 * X[rows, cols] - p.val
    return 0.25 * float(r @ r) + lam * float(np.trace(X))


def qsdp_fd_gradient(p, X, lam, h=1e-3):
    """Gradient of f + lam tr on symmetric matrices by central differences
    (exact up to rounding: the objective is quadratic in X).  For E symmetric,
    <G, E> = D phi[E]: E = e_a e_a^T gives G_aa, E = e_a e_b^T + e_b e_a^T gives 2 G_ab."""
    n = X.shape[0]
    G = np.zeros((n, n))
    for a in range(n):
        for b in range(a, n):
            E = np.zeros((n, n))
            E[a, b] = E[b, a] = 1.0
            d = (qsdp_dense_f(p, X + h * E, lam) - qsdp_dense_f(p, X - h * E, lam)) / (2 * h)
            G[a, b] = G[b, a] = d if a == b else 0.5 * d
    return G


def reduced_projection(Z):
    """Projection onto {X psd, <E, X> = 0} = {Q Y Q^T : Y psd}, Q an orthonormal
    basis of the complement of e: Q P_S+(Q^T Z Q) Q^T (no use of Lemma PiX)."""
    n = Z.shape[0]
    Q = np.linalg.svd(np.eye(n) - np.ones((n, n)) / n)[0][:, :n - 1]
    w, V = np.linalg.eigh(Q.T @ (0.5 * (Z + Z.T)) @ Q)
    return Q @ ((V * np.maximum(w, 0.0)) @ V.T) @ Q.T


QSDP_CASES = [(10, 6, 0.7, 0.3), (12, 8, 2.0, 1.2), (9, 4, 0.2, 0.05)]


def _qsdp_parts(case):
    n, deg, lam, scale = case
    p = synth.rke(n, deg, seed=n + deg)
    W = rke.center(scale * rand((n, 3), n))
    X = W @ W.T
    r = rke.pair_residual(p, W)
    G = qsdp_fd_gradient(p, X, lam)
    return p, W, X, r, G, lam


def qsdp_grad_pin_holds(grad_norm_fn, rtol=1e-8):
    for case in QSDP_CASES:
        p, W, X, r, G, lam = _qsdp_parts(case)
        if not math.isclose(grad_norm_fn(p, r, lam), np.linalg.norm(G), rel_tol=rtol):
            return False
    return True


def test_qsdp_grad_norm_matches_finite_difference_gradient():
    """grad_norm = ||grad (f + lam tr)(X~)||_F with the gradient from central
    differences of the dense objective (pairs counted once, off-diagonal
    entries -r_ij on both sides of the diagonal)."""
    assert qsdp_grad_pin_holds(rke.grad_norm)
    for case in QSDP_CASES:   # and the gradient is L_r + lam I with e in its kernel up to lam
        p, W, X, r, G, lam = _qsdp_parts(case)
        assert np.allclose(G @ np.ones(p.n), lam * np.ones(p.n), atol=1e-7)


def _grad_slip(kind):
    def fn(p, r, lam):
        deg = np.bincount(p.rows(), weights=r, minlength=p.n)
        if kind == "doubled_off_diagonal":
            return float(np.sqrt(np.sum((deg + lam) ** 2) + 2.0 * np.dot(r, r)))
        if kind == "no_lambda":
            return float(np.sqrt(np.sum(deg ** 2) + np.dot(r, r)))
        if kind == "absolute_degrees":
            ad = np.bincount(p.rows(), weights=np.abs(r), minlength=p.n)
            return float(np.sqrt(np.sum((ad + lam) ** 2) + np.dot(r, r)))
        if kind == "lambda_everywhere":
            return float(np.sqrt(np.sum((deg + lam) ** 2) + np.sum((r + lam) ** 2)))
        raise ValueError(kind)
    return fn


@pytest.mark.parametrize("kind", ["doubled_off_diagonal", "no_lambda", "absolute_degrees",
                                  "lambda_everywhere"])
def test_qsdp_grad_pin_rejects_planted_slips(kind):
    assert not qsdp_grad_pin_holds(_grad_slip(kind))


def qsdp_stop_pin_holds(stop_fn, rtol=1e-8):
    """stop_fn(p, W~, W+, r, alpha, lam) against the dense prox-gradient mapping
    with the exact projection (reduced coordinates) and the finite-difference
    gradient, at the solver's step alpha = 1.99 / (2 + 2 max degree)."""
    for case in QSDP_CASES:
        p, W, X, r, G, lam = _qsdp_parts(case)
        alpha = 1.99 / (2.0 + 2.0 * float(np.diff(p.row_ptr).max()))
        Xp = reduced_projection(X - alpha * G)
        w, V = np.linalg.eigh(Xp)
        keep = w > 1e-12 * max(w.max(), 1.0)
        Wn = V[:, keep] * np.sqrt(w[keep])
        expect = np.linalg.norm(X - Xp) / (alpha * (1.0 + np.linalg.norm(X) + np.linalg.norm(G)))
        if not math.isclose(stop_fn(p, W, Wn, r, alpha, lam), expect, rel_tol=rtol):
            return False
    return True


def test_qsdp_stop_residual_matches_dense_prox_gradient_mapping():
    assert qsdp_stop_pin_holds(rke.stop_residual)


def test_qsdp_stop_residual_of_the_oracle_pg_step():
    """The PG step the oracle's solve takes (eig_prox from a full start block)
    fed to stop_residual gives the dense value too."""
    for case in QSDP_CASES:
        p, W, X, r, G, lam = _qsdp_parts(case)
        alpha = 1.99 / rke.lipschitz_bound(p)
        ep = rke.eig_prox(p, W, r, alpha, lam, rand((p.n, p.n), 5), 1e-15, max_iter=5000)
        Xp = reduced_projection(X - alpha * G)
        expect = np.linalg.norm(X - Xp) / (alpha * (1.0 + np.linalg.norm(X) + np.linalg.norm(G)))
        assert math.isclose(rke.stop_residual(p, W, ep.W, r, alpha, lam), expect, rel_tol=1e-7)


def _stop_slip(kind):
    def fn(p, W, Wn, r, alpha, lam):
        d = math.sqrt(core.diff_fro2_split(W, W, Wn, Wn))
        x = math.sqrt(core.fro2_factored(W, W))
        g = rke.grad_norm(p, r, lam)
        if kind == "no_alpha":
            return d / (1.0 + x + g)
        if kind == "no_one":
            return d / (alpha * (x + g))
        if kind == "squared_norms":
            return d / (alpha * (1.0 + x * x + g * g))
        if kind == "alpha_squared":
            return d / (alpha * alpha * (1.0 + x + g))
        raise ValueError(kind)
    return fn


@pytest.mark.parametrize("kind", ["no_alpha", "no_one", "squared_norms", "alpha_squared"])
def test_qsdp_stop_pin_rejects_planted_slips(kind):
    assert not qsdp_stop_pin_holds(_stop_slip(kind))


def test_lipschitz_bound_dominates_the_operator_norm():
    """||A^* A||_2 from the explicit pair matrix (one row per pair, entries
    +1, +1, -1, -1 at X_ii, X_jj, X_ij, X_ji over symmetric X) never exceeds
    lipschitz_bound, and the bound is within a factor 2 + 2 max deg of it."""
    for n, deg, seed in ((12, 6, 2), (20, 10, 3)):
        p = synth.rke(n, deg, seed=seed)
        rows, cols = p.rows(), p.col
        pairs = [(i, j) for i, j in zip(rows, cols) if i < j]
        # coordinates of a symmetric X: the n diagonal entries and each X_ij = X_ji (i < j)
        # scaled by sqrt(2) so the Frobenius inner product is the Euclidean one
        idx = {}
        for a in range(n):
            idx[(a, a)] = len(idx)
        for a in range(n):
            for b in range(a + 1, n):
                idx[(a, b)] = len(idx)
        Amat = np.zeros((len(pairs), len(idx)))
        for t, (i, j) in enumerate(pairs):
            Amat[t, idx[(i, i)]] = 1.0
            Amat[t, idx[(j, j)]] = 1.0
            Amat[t, idx[(i, j)]] = -2.0 / math.sqrt(2.0)
        nrm = np.linalg.norm(Amat, 2) ** 2
        assert nrm <= rke.lipschitz_bound(p) * (1 + 1e-12)
        assert nrm >= 4.0 - 1e-12   # one pair alone: ||A_p||^2 = 1 + 1 + 2
