"""BM-Global for the regularized kernel estimation QSDP: plain FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY: imported by tests, never by the product path.
Shares no code with the GPU library.

Problem (QSDP section, eq. QSDP with unit weights):
    min  f(X) + lam tr(X)   over X positive semidefinite with <E, X> = 0,
    f(X) = 1/2 sum over pairs (i, j) in Omega of (X_ii + X_jj - 2 X_ij - d_ij^2)^2.
Omega is stored symmetrically (both (i, j) and (j, i), value d_ij^2), so a sum
over stored entries counts every pair twice.

BM form (eq. bm2 / eq. bmprob): X = W W^T with W n x k and W^T e = 0,
    F~(W) = f(W W^T) + lam ||W||_F^2      (tr(W W^T) = ||W||_F^2).

Function -> passage -> pin (tests/test_oracle_rke.py):
  pair_residual, lap_apply   A(X) - b and A^*(r) = L_r (the Laplacian with edge
                             weights r)          -> dense A, A^* on tiny inputs
  bm_phase, quartic_step     BM phase, eq. nonincrease: nonlinear conjugate
                             gradient with exact (quartic) line search (reading)
                             -> the step against a fine grid, monotone F~
  project_dense              Lemma PiX: P_X(G) = P_S+(J G J)
                             -> Dykstra's alternating projections
  eig_prox                   the PG step's eigen-decomposition by block
                             subspace iteration (reading)   -> dense eigh
  grad_norm, stop_residual   ||grad f~||_F and the stop residual (prox-gradient
                             mapping)  -> finite-difference gradient of the dense
                             objective, projection in reduced coordinates
  lipschitz_bound            step size bound on ||A^* A|| -> dense operator norm
  solve                      Algorithm 1 on this problem    -> dense proximal
                             gradient with the exact projection
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np

from . import core, rng


def pair_residual(prob, W) -> np.ndarray:
    """r_p = ||w_i - w_j||^2 - d_ij^2 = (A(W W^T) - b)_p for every stored entry."""
    if W.shape[1] == 0:
        return -prob.val.copy()
    D = W[prob.rows()] - W[prob.col]
    return np.sum(D * D, axis=1) - prob.val


def lap_apply(prob, r, U) -> np.ndarray:
    """A^*(r) U = L_r U, L_r = sum over pairs r_ij (e_i - e_j)(e_i - e_j)^T:
    (L_r U)_i = sum_j r_ij (u_i - u_j) over the stored row i."""
    deg = np.bincount(prob.rows(), weights=r, minlength=prob.n)
    return deg[:, None] * U - core.spmm(prob, r, U)


def bm_objective(prob, W, lam: float) -> float:
    """F~(W) = 1/2 sum over pairs r^2 + lam ||W||^2 (stored entries count twice)."""
    r = pair_residual(prob, W)
    return 0.25 * float(np.dot(r, r)) + lam * float(np.sum(W * W))


def center(V) -> np.ndarray:
    """J V with J = I - e e^T / n (removes the column means)."""
    return V - V.mean(axis=0) if V.shape[1] else V


def quartic_step(prob, W, D, r, lam: float) -> float:
    """Exact line search of F~ along D from W (residual r at W): along W + t D each
    pair's squared distance is a0 + 2 t a1 + t^2 a2 with a1 = (w_i - w_j).(d_i - d_j)
    and a2 = ||d_i - d_j||^2, so F~ is a quartic in t; its exact minimiser over
    t >= 0."""
    rows, cols = prob.rows(), prob.col
    dW, dD = W[rows] - W[cols], D[rows] - D[cols]
    a1 = np.sum(dW * dD, axis=1)
    a2 = np.sum(dD * dD, axis=1)
    # sums over stored entries are twice the sums over pairs
    c1 = float(np.dot(r, a1)) + 2.0 * lam * float(np.sum(W * D))
    c2 = float(np.dot(a1, a1)) + 0.5 * float(np.dot(r, a2)) + lam * float(np.sum(D * D))
    c3 = float(np.dot(a1, a2))
    c4 = 0.25 * float(np.dot(a2, a2))
    return core.quartic_min(c1, c2, c3, c4)


def bm_phase(prob, W, lam: float, steps: int):
    """The BM phase (reading; the paper runs a Riemannian solver, and the
    constraint W^T e = 0 is a linear subspace here): `steps` steps of nonlinear
    conjugate gradient (Polak-Ribiere with restart at negative beta or a
    non-descent direction) on F~ with the exact quartic line search, starting
    from steepest descent.  G = L_r W + lam W is half the gradient of F~ and
    keeps e^T G = 0 (J applied against rounding).  F~ never increases
    (eq. nonincrease).  Returns (W, list of steps t)."""
    G_prev, D, ts = None, None, []
    for _ in range(steps):
        r = pair_residual(prob, W)
        G = center(lap_apply(prob, r, W) + lam * W)
        if G_prev is None:
            D = -G
        else:
            beta = max(0.0, float(np.sum(G * (G - G_prev))) / float(np.sum(G_prev * G_prev)))
            D = -G + beta * D
            if float(np.sum(D * G)) >= 0.0:
                D = -G
        t = quartic_step(prob, W, D, r, lam)
        W = W + t * D
        G_prev = G
        ts.append(t)
    return W, ts


def lipschitz_bound(prob) -> float:
    """||A^* A|| <= 2 + 2 max_i deg(i) (Gershgorin on the Gram matrix of the
    pair matrices (e_i - e_j)(e_i - e_j)^T: 4 on the diagonal, 1 for pairs
    sharing an object)."""
    deg = np.diff(prob.row_ptr)
    return 2.0 + 2.0 * float(deg.max() if deg.size else 0)


def project_dense(G) -> np.ndarray:
    """Lemma PiX: the projection onto {X psd, <E, X> = 0} is P_S+(J G J)."""
    n = G.shape[0]
    J = np.eye(n) - np.ones((n, n)) / n
    w, V = np.linalg.eigh(J @ (0.5 * (G + G.T)) @ J)
    w = np.maximum(w, 0.0)
    return (V * w) @ V.T


@dataclass
class EigResult:
    W: np.ndarray          # U_+ sqrt(theta_+): the new factor
    U: np.ndarray          # eigenvectors kept
    theta: np.ndarray      # all Ritz values of the last basis
    iters: int
    u: object = None       # Ritz vector of the largest Ritz value not kept (None if all kept)


def eig_prox(prob, W, r, alpha: float, lam: float, U0, tau: float, max_iter: int = 50,
             p: int = 0, tau_new: float = 0.0) -> EigResult:
    """Prox of the PG step from X~ = W W^T (Lemma PiX):
        X+ = P_S+(M),  M = J (X~ - alpha (L_r + lam I)) J = X~ - alpha L_r - alpha lam J
    (J X~ J = X~ as W^T e = 0, and J L_r J = L_r).  Reading: Algorithm 2 (LmSVD)
    with history length p on the shifted operator L = M + sigma I, sigma =
    alpha (2 max_i sum_j |r_ij| + lam), which is positive semidefinite
    (Gershgorin), so the iteration finds the algebraically largest eigenvalues
    of M.  With q the width of the start block U = orth(J U0) and Y = M U:
      the block subspace is ran(U^{i}, ..., U^{i-p'}), p' = min(p, i), with the
      orthonormal basis Q = [U, P S] of eqs. PUi and orth-W (P the history
      blocks projected onto ker(U^T), S over the eigenvalues of P^T P above
      core.LMSVD_EIG_TOL), and M Q = [Y, (Y_old - Y C) S] from products already
      made (C = U^T U_old);
      Rayleigh-Ritz on M over Q (the eigenvectors of L, values shifted by
      sigma): theta, V = the q leading eigenpairs of Q^T M Q (eq. lmsvd-opt);
      next U = orth(J L(Q V)) = orth(J (M Q V + sigma Q V)), Y = M U.
    With p = 0, Q = U and this is the block subspace iteration with a
    Rayleigh-Ritz rotation.  Stop once the Ritz values above 0, the largest and
    the first one not above 0 moved by at most tau * |largest| (the last so that
    a positive eigenvalue still being approached is not cut off).  Reading, with
    history (p >= 1) and tau_new > 0: the newest of those values (the first one
    not above 0, or the smallest above 0 when all are) is held to
    max(tau |largest|, min(tau_new, 1e-4 |largest|)) instead, tau_new being an
    absolute tolerance the caller ties to the size of the PG step; it sits in
    the cluster of small eigenvalues of the complement, where the test
    relative to the largest would wait for far more accuracy than the step's
    own size calls for (the error this admits in X+ is of the order of tau_new,
    the relative inexactness of eq. inexact).  The output is the last
    Rayleigh-Ritz step's: X+ = (Q V_+) diag(theta_+) (Q V_+)^T, and u = Q
    v_{k+1}, the Ritz vector of the largest Ritz value not kept."""
    n = prob.n
    absdeg = np.bincount(prob.rows(), weights=np.abs(r), minlength=n)
    sigma = alpha * (2.0 * float(absdeg.max() if absdeg.size else 0.0) + lam)

    def apply_M(U):
        out = -alpha * lap_apply(prob, r, U) - alpha * lam * center(U)
        if W.shape[1]:
            out += W @ (W.T @ U)
        return out

    U = core.orth(center(U0))
    if U.shape[1] == 0:
        return EigResult(np.zeros((n, 0)), np.zeros((n, 0)), np.zeros(0), 0)
    Y = apply_M(U)
    hist = []                     # (U^{j}, M U^{j}) for j = i-1, ..., i-p'
    prev = None
    it = 0
    for it in range(1, max_iter + 1):
        q = U.shape[1]
        Q, MQ = U, Y
        if hist:
            Uold = np.column_stack([h[0] for h in hist])
            Yold = np.column_stack([h[1] for h in hist])
            C = U.T @ Uold
            Pm = Uold - U @ C                                  # eq. PUi
            lp, Ut = core.eigh_desc(Pm.T @ Pm)
            keep = lp > core.LMSVD_EIG_TOL
            S = Ut[:, keep] / np.sqrt(lp[keep])
            Q = np.column_stack([U, Pm @ S])                   # eq. orth-W
            MQ = np.column_stack([Y, (Yold - Y @ C) @ S])
        theta, V = core.eigh_desc(Q.T @ MQ)
        theta, V = theta[:q], V[:, :q]                         # eq. lmsvd-opt
        done = False
        if prev is not None and prev.size == theta.size and theta.size:
            J = theta > 0.0
            J[0] = True
            jn = min(int(np.sum(theta > 0.0)), theta.size - 1)         # the first one not kept
            J[jn] = True
            lim = tau * abs(theta[0])
            if p > 0 and tau_new > 0.0 and jn > 0:
                J[jn] = False
                lim_new = max(lim, min(tau_new, 1e-4 * abs(theta[0])))
                done = (float(np.max(np.abs(theta[J] - prev[J]))) <= lim
                        and abs(theta[jn] - prev[jn]) <= lim_new)
            else:
                done = float(np.max(np.abs(theta[J] - prev[J]))) <= lim
        prev = theta
        if done or it == max_iter:
            break
        Unew = core.orth(center(MQ @ V + sigma * (Q @ V)))
        if p > 0:
            hist = ([(U, Y)] + hist)[:p]
        U = Unew
        if U.shape[1] == 0:
            return EigResult(np.zeros((n, 0)), np.zeros((n, 0)), np.zeros(0), it)
        Y = apply_M(U)
    keep = theta > 0.0
    kp = int(np.sum(keep))
    Up = Q @ V[:, :kp]
    u = Q @ V[:, kp] if kp < theta.size else None
    return EigResult(Up * np.sqrt(theta[:kp]), Up, theta, it, u)


@dataclass
class RkeRecord:
    t: int
    F: float
    residual: float
    k: int
    ssi_iters: int


@dataclass
class RkeResult:
    W: np.ndarray
    k: int
    F: float
    residual: float
    iters: int
    converged: bool
    history: List[RkeRecord] = field(default_factory=list)


def objective(prob, W, lam: float) -> float:
    """F(X) = f(X) + lam tr(X) at X = W W^T (W^T e = 0 assumed)."""
    return bm_objective(prob, W, lam)


def grad_norm(prob, r, lam: float) -> float:
    """||L_r + lam I||_F: diagonal deg_i + lam, off-diagonal -r_ij per stored entry."""
    deg = np.bincount(prob.rows(), weights=r, minlength=prob.n)
    return float(np.sqrt(np.sum((deg + lam) ** 2) + np.dot(r, r)))


def step_norm(W, Wn) -> float:
    """||W W^T - Wn Wn^T||_F, split over ran(W) and its complement
    (core.diff_fro2_split) so that nothing cancels."""
    if W.shape[1]:
        return float(np.sqrt(core.diff_fro2_split(W, W, Wn, Wn)))
    return float(np.sqrt(core.fro2_factored(Wn, Wn)))


def stop_residual(prob, W, Wn, r, alpha: float, lam: float) -> float:
    """Stop residual of the PG step from X~ = W W^T (residual r) to X+ = Wn Wn^T:
        ||X~ - X+||_F / (alpha (1 + ||X~||_F + ||grad f~(X~)||_F)),
    grad f~ = L_r + lam I (grad_norm).  ||X~ - X+|| / alpha is the norm of the
    prox-gradient mapping at step alpha (the QSDP optimality measure of Sec. 6.2
    uses the prox at unit step; alpha is far below 1 here, so the step itself
    would stop far too early); the difference is split over ran(W) and its
    complement (diff_fro2_split) so that nothing cancels."""
    d = step_norm(W, Wn)
    return float(d / (alpha * (1.0 + np.sqrt(core.fro2_factored(W, W)) + grad_norm(prob, r, lam))))


def solve(prob, lam: float, k0: int = 8, tol: float = 1e-6, max_iter: int = 500, bm_epochs: int = 10,
          ssi_max_iter: int = 50, ssi_tol_floor: float = 1e-12, seed: int = 0,
          alpha_scale: float = 1.99, lmsvd_p: int = 0, psi0: float = 0.1, callback=None) -> RkeResult:
    """Algorithm 1 on the QSDP (readings as in eig_prox and bm_phase):
    alpha = alpha_scale / (2 + 2 max degree); the first step from X_{-1} = 0
    starts the subspace iteration from J times a Gaussian n x k0 block (stream
    STREAM_SKETCH); then per outer iteration a BM phase of bm_epochs conjugate
    gradient steps (bm_phase) and the PG step (eig_prox with history lmsvd_p),
    warm-started from [Ubase, u_t + xi_t] with Ubase = orth(J W~_t) and the
    rank safeguard column of eq. rt (core.safeguard_column, stream
    STREAM_SAFEGUARD + t): u is the Ritz vector of the largest Ritz value not
    kept at the latest PG step that truncated one, xi_t a random vector of
    norm psi_t orthogonal to [Ubase, u_t]; psi starts at psi0 and halves after
    every PG step that truncates exactly one Ritz value (Suppl. A.1.3); the
    newest Ritz value's tolerance tau_new of eig_prox is a tenth of the
    previous PG step's ||X~ - X+||_F (with history only).  The
    rank grows by at most one per step (reading: far from the optimum nearly
    every eigenvalue of the PG point is positive, and a block orth([U_t, W~_t])
    doubles), and the rank update k = number of positive Ritz values.  Stop
    when ||X~ - X+||_F / (alpha (1 + ||X~||_F + ||grad f~(X~)||_F)) <= tol: the
    prox-gradient mapping, as alpha is far below 1 here (the tolerance of the
    subspace iteration tightens with that residual)."""
    n = prob.n
    alpha = alpha_scale / lipschitz_bound(prob)
    Om = rng.normals(seed, rng.STREAM_SKETCH, n * k0).reshape(n, k0)
    e0 = eig_prox(prob, np.zeros((n, 0)), -prob.val, alpha, lam, Om, 1e-4, ssi_max_iter, lmsvd_p)
    W = e0.W
    u_keep = e0.u
    psi = psi0
    hist: List[RkeRecord] = []
    res, res_prev, conv, t = np.inf, 1.0, False, 0
    step_prev = 0.0
    F = objective(prob, W, lam)
    for t in range(max_iter):
        if W.shape[1] and bm_epochs > 0:
            W, _ = bm_phase(prob, W, lam, bm_epochs)
        r = pair_residual(prob, W)
        tau = max(ssi_tol_floor, min(1e-4, 0.1 * res_prev * res_prev))
        Ubase = core.orth(center(W)) if W.shape[1] else np.zeros((n, 0))
        col = core.safeguard_column(Ubase, u_keep, psi, seed, t)
        ep = eig_prox(prob, W, r, alpha, lam, np.column_stack([Ubase, col]), tau, ssi_max_iter, lmsvd_p,
                      0.1 * step_prev)
        res = stop_residual(prob, W, ep.W, r, alpha, lam)
        step_prev = step_norm(W, ep.W)
        # safeguard bookkeeping (eq. rt)
        trunc = ep.theta.size - ep.W.shape[1]
        u_keep = ep.u if trunc >= 1 else None
        if trunc == 1:
            psi *= 0.5
        W = ep.W
        F = objective(prob, W, lam)
        rec = RkeRecord(t, F, res, W.shape[1], ep.iters)
        hist.append(rec)
        if callback:
            callback(rec)
        res_prev = res
        if res <= tol:
            conv = True
            break
    return RkeResult(W, W.shape[1], F, res, t + 1, conv, hist)
