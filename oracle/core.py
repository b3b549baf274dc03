"""BM-Global for nuclear-norm matrix completion: plain FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the CPU
baseline of the benchmark, never by the product path.  Shares no code with the
GPU library.

Problem (MC), Sec. 1:   min_X  1/2 ||P_Omega(X - A)||_F^2 + lambda ||X||_*
BM form (MF)/(BM-nuclear), Sec. 1-2:
        min_{W,H}  1/2 ||P_Omega(W H^T - A)||_F^2 + lambda/2 (||W||_F^2 + ||H||_F^2)

Function -> passage it follows -> what pins it (tests/test_oracle_*.py):

  sddmm / spmm / spmm_t   MC gradient P_Omega(X - A) is sparse (Sec. 5.1)
                          -> brute force on masked dense matrices
  nuclear_norm            Lemma "equivalent" (Sec. 2)       -> dense SVD; balanced factors
  bm_epoch                BM phase + non-increase condition (Sec. 3, eq. nonincrease);
                          solver = preconditioned steepest descent, exact line search (reading)
                          -> brute-force minimisation of the 1-D quadratic; monotone F~
  polymf_epoch            polyMF-SS (Sec. 6.1.1): column-pair BCD, exact quartic line search
                          -> quartic coefficients against the dense block objective; the
                             step against a fine grid; monotone F~ per block; solves reach
                             the dense optimum
  orth                    range basis used by eq-ssi, eq. rt0, eq. rt      -> span tests
  lmsvd                   Algorithm 2, history length p_t >= 0 (Suppl. A.1.2)
                          -> dense eigendecomposition of Z Z^T; Ritz values against the
                             dense compression of Z Z^T onto an SVD basis of the subspace;
                             fewer iterations with history on a slow spectrum
  prox_from_basis         eqs. exactSVD, approxSVD, truncate (Suppl. A.1.1)
                          -> full SVD + soft-threshold (eq. proxnuc) when the basis spans ran(Z)
  initialize              HMT + Nystrom, eq. nys (Suppl. A.1.4)
                          -> exact prox of P_Omega(A) when k0 >= rank
  safeguard_column        eq. rt and the noise schedule (Suppl. A.1.3)  -> orthogonality / norm checks
  step_norm / residual    prox-gradient residual ||X~ - X+|| in factored form
                          -> dense computation on small inputs; eq. trace (Suppl. B.1,
                             sign corrected) as a second route
  solve                   Algorithm 1 with x = 1 PG step per y = 3 BM epochs (Sec. 6.1.1)
                          -> full-Omega closed form SVT_lambda(A); dense proximal gradient to
                             1e-12; duality gap certificate; optimality conditions
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.linalg
from threadpoolctl import threadpool_limits

from . import rng

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c (plain C, OpenMP over independent rows)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp,
                               os.path.join(_HERE, "oracle.c")])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        i64, p, ci = ctypes.c_int64, ctypes.c_void_p, ctypes.c_int
        lib.orc_sddmm.argtypes = [i64, p, p, p, ci, p, i64, p, i64, p]
        lib.orc_sddmm.restype = None
        lib.orc_spmm.argtypes = [i64, p, p, p, ci, p, i64, p, i64]
        lib.orc_spmm.restype = None
        lib.orc_spmm_t.argtypes = [i64, i64, p, p, p, ci, p, i64, p, i64]
        lib.orc_spmm_t.restype = None
        lib.orc_sumsq_rows.argtypes = [i64, p, p]
        lib.orc_sumsq_rows.restype = ctypes.c_double
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


# ----------------------------------------------------------------------------- Omega

@dataclass
class Omega:
    """Omega in CSR form with the observed values (any object with these
    fields works as a problem for this module)."""
    m: int
    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def rows(self) -> np.ndarray:
        return np.repeat(np.arange(self.m, dtype=np.int64), np.diff(self.row_ptr))


def transpose(prob) -> Omega:
    """Omega of A^T (entries re-sorted by column, then row)."""
    rows = np.repeat(np.arange(prob.m, dtype=np.int64), np.diff(prob.row_ptr))
    order = np.lexsort((rows, prob.col))
    rp = np.zeros(prob.n + 1, np.int64)
    np.cumsum(np.bincount(prob.col, minlength=prob.n), out=rp[1:])
    return Omega(prob.n, prob.m, rp, rows[order].astype(np.int32), np.asarray(prob.val)[order])


# ----------------------------------------------------------------------------- sparse loops

def sddmm(prob, X: np.ndarray, Y: np.ndarray, with_values: bool = True) -> np.ndarray:
    """R[p] = x_i . y_j - A_ij over Omega (A taken as 0 if ``with_values`` is False).
    At X = W, Y = H this is grad f(W H^T) = P_Omega(W H^T - A) (MC, Sec. 5.1)."""
    X, Y = _c(X), _c(Y)
    k = X.shape[1]
    assert Y.shape[1] == k
    R = np.empty(prob.nnz, np.float64)
    if prob.nnz == 0:
        return R
    _load().orc_sddmm(prob.m, _p(prob.row_ptr), _p(prob.col), _p(prob.val) if with_values else None,
                      k, _p(X), max(k, 1), _p(Y), max(k, 1), _p(R))
    return R


def spmm(prob, S: np.ndarray, B: np.ndarray) -> np.ndarray:
    """C = S B with S the sparse m x n matrix with values S on Omega, B n x q."""
    B = _c(B)
    q = B.shape[1]
    C = np.zeros((prob.m, q), np.float64)
    if q == 0 or prob.nnz == 0:
        return C
    _load().orc_spmm(prob.m, _p(prob.row_ptr), _p(prob.col), _p(_c(S)), q, _p(B), q, _p(C), q)
    return C


def spmm_t(prob, S: np.ndarray, B: np.ndarray) -> np.ndarray:
    """C = S^T B with B m x q (C is n x q)."""
    B = _c(B)
    q = B.shape[1]
    C = np.zeros((prob.n, q), np.float64)
    if q == 0 or prob.nnz == 0:
        return C
    _load().orc_spmm_t(prob.m, prob.n, _p(prob.row_ptr), _p(prob.col), _p(_c(S)), q, _p(B), q,
                       _p(C), q)
    return C


def sumsq(prob, R: np.ndarray) -> float:
    if prob.nnz == 0:
        return 0.0
    return float(_load().orc_sumsq_rows(prob.m, _p(prob.row_ptr), _p(_c(R))))


# ----------------------------------------------------------------------------- objectives

def nuclear_norm(W: np.ndarray, H: np.ndarray) -> float:
    """||W H^T||_* without forming the product: W = Q_W R_W, H = Q_H R_H, so the
    singular values of W H^T are those of R_W R_H^T (k x k)."""
    if W.shape[1] == 0:
        return 0.0
    _, Rw = np.linalg.qr(W)
    _, Rh = np.linalg.qr(H)
    return float(np.linalg.svd(Rw @ Rh.T, compute_uv=False).sum())


def loss(prob, W, H):
    """f(W H^T) = 1/2 ||P_Omega(W H^T - A)||^2 and the residual values R."""
    R = sddmm(prob, W, H)
    return 0.5 * sumsq(prob, R), R


def objective(prob, W, H, lam: float) -> float:
    """F(X) of (MC) at X = W H^T."""
    f, _ = loss(prob, W, H)
    return f + lam * nuclear_norm(W, H)


def bm_objective(prob, W, H, lam: float) -> float:
    """F~(W, H) of (BM-nuclear) / (MF)."""
    f, _ = loss(prob, W, H)
    return f + 0.5 * lam * (float(np.sum(W * W)) + float(np.sum(H * H)))


# ----------------------------------------------------------------------------- BM phase

def _precond(F: np.ndarray, lam: float) -> np.ndarray:
    """(F^T F + lambda I)^{-1}: the k x k scaling of the preconditioned gradient
    step (Remark on the BM solver: preconditioned gradient-type methods)."""
    k = F.shape[1]
    return np.linalg.inv(F.T @ F + lam * np.eye(k))


def bm_half_step_W(prob, W, H, lam):
    """One preconditioned steepest-descent step on W of (MF), exact line search.

    Gradient G = R H + lambda W with R = P_Omega(W H^T - A); direction
    D = -G (H^T H + lambda I)^{-1}.  Along W + s D the objective is the quadratic
        1/2 ||R + s P_Omega(D H^T)||^2 + lambda/2 ||W + s D||^2 + const,
    minimised at s = -<G, D> / (||P_Omega(D H^T)||^2 + lambda ||D||^2)."""
    R = sddmm(prob, W, H)
    G = spmm(prob, R, H) + lam * W
    D = -G @ _precond(H, lam)
    gd = -float(np.sum(G * D))
    if gd <= 0.0:
        return W.copy(), 0.0
    C = sddmm(prob, D, H, with_values=False)
    s = gd / (sumsq(prob, C) + lam * float(np.sum(D * D)))
    return W + s * D, s


def bm_half_step_H(prob, W, H, lam):
    """Same on H: G = R^T W + lambda H, D = -G (W^T W + lambda I)^{-1},
    curvature ||P_Omega(W D^T)||^2 + lambda ||D||^2."""
    R = sddmm(prob, W, H)
    G = spmm_t(prob, R, W) + lam * H
    D = -G @ _precond(W, lam)
    gd = -float(np.sum(G * D))
    if gd <= 0.0:
        return H.copy(), 0.0
    C = sddmm(prob, W, D, with_values=False)
    s = gd / (sumsq(prob, C) + lam * float(np.sum(D * D)))
    return H + s * D, s


def bm_epoch(prob, W, H, lam):
    """One epoch of the BM-phase solver: a W step then an H step.  Each step
    minimises F~ exactly along a descent direction, so F~ never increases (the
    only requirement on the BM phase, Sec. 3 eq. nonincrease)."""
    W1, sw = bm_half_step_W(prob, W, H, lam)
    H1, sh = bm_half_step_H(prob, W1, H, lam)
    return W1, H1, (sw, sh)


# ----------------------------------------------------------------------------- polyMF-SS BM solver

def quartic_min(c1: float, c2: float, c3: float, c4: float) -> float:
    """Global minimiser over t >= 0 of psi(t) = c1 t + c2 t^2 + c3 t^3 + c4 t^4
    (c4 >= 0): the best of t = 0 and the positive real roots of psi'."""
    cands = [0.0]
    for r in np.roots([4.0 * c4, 3.0 * c3, 2.0 * c2, c1]):
        if abs(r.imag) <= 1e-9 * max(1.0, abs(r.real)) and r.real > 0.0:
            cands.append(float(r.real))
    psi = lambda t: ((c4 * t + c3) * t + c2) * t * t + c1 * t  # noqa: E731
    return min(cands, key=lambda t: (psi(t), t))


def polymf_block(prob, W, H, j: int, lam: float, R):
    """One block of the polyMF-SS BM solver (Sec. 6.1.1: block coordinate
    descent with exact line search, a block being column j of W and of H).

    On the block, phi(w, h) = 1/2 ||P_Omega(R - w_j h_j^T + w h^T)||^2
    + lam/2 (||w||^2 + ||h||^2).  Direction (reading): the block gradient
        g_w = R h_j + lam w_j,   g_h = R^T w_j + lam h_j
    scaled entrywise by the diagonal of the block Hessian of each half,
        d_w[i] = -g_w[i] / (sum_{l in Omega_i} h_l^2 + lam)   (and likewise d_h),
    so that t = 1 is the exact minimiser when only one half moves.  Along
    (w + t d_w, h + t d_h) every sampled residual is r + t a + t^2 b with
        a = d_w[i] h_l + w_i d_h[l],   b = d_w[i] d_h[l],
    so phi is a quartic in t; the step is its exact minimiser over t >= 0.
    Returns (W, H, R, t) with the residual R updated on Omega."""
    rows, cols = prob.rows(), prob.col
    w, h = W[:, j].copy(), H[:, j].copy()
    ones = np.ones(prob.nnz)
    gw = spmm(prob, R, h[:, None])[:, 0] + lam * w
    gh = spmm_t(prob, R, w[:, None])[:, 0] + lam * h
    cw = spmm(prob, ones, (h * h)[:, None])[:, 0] + lam
    ch = spmm_t(prob, ones, (w * w)[:, None])[:, 0] + lam
    dw, dh = -gw / cw, -gh / ch
    a = dw[rows] * h[cols] + w[rows] * dh[cols]
    b = dw[rows] * dh[cols]
    c1 = float(np.dot(R, a)) + lam * (float(np.dot(w, dw)) + float(np.dot(h, dh)))
    c2 = 0.5 * float(np.dot(a, a)) + float(np.dot(R, b)) \
        + 0.5 * lam * (float(np.dot(dw, dw)) + float(np.dot(dh, dh)))
    c3 = float(np.dot(a, b))
    c4 = 0.5 * float(np.dot(b, b))
    t = quartic_min(c1, c2, c3, c4)
    W, H = W.copy(), H.copy()
    W[:, j] = w + t * dw
    H[:, j] = h + t * dh
    return W, H, R + t * a + t * t * b, t


def polymf_epoch(prob, W, H, lam):
    """One polyMF-SS epoch: blocks j = 0, ..., k-1 in order, from the residual
    of the incoming factors.  F~ never increases (eq. nonincrease)."""
    R = sddmm(prob, W, H)
    steps = []
    for j in range(W.shape[1]):
        W, H, R, t = polymf_block(prob, W, H, j, lam, R)
        steps.append(t)
    return W, H, steps


# ----------------------------------------------------------------------------- linear algebra helpers

ORTH_TOL = 1e-6      # relative singular-value cut of orth() on unit-norm columns


def orth(M: np.ndarray, tol: float = ORTH_TOL) -> np.ndarray:
    """Orthonormal basis of ran(M) (the orth() of eq-ssi, eq. rt0 and eq. rt).

    Columns are first scaled to unit norm (the range is unchanged and the
    numerical-rank cut no longer depends on column scaling) and zero columns
    dropped; a column-pivoted QR (LAPACK geqp3) then picks columns greedily by
    largest remaining norm, and the basis keeps the first r of them, r being
    the number of pivots with |R_jj| > tol."""
    if M.ndim != 2 or M.shape[1] == 0:
        return np.zeros((M.shape[0], 0))
    nrm = np.linalg.norm(M, axis=0)
    keep = nrm > 0
    if not keep.any():
        return np.zeros((M.shape[0], 0))
    Mn = M[:, keep] / nrm[keep]
    Q, R, _ = scipy.linalg.qr(Mn, mode="economic", pivoting=True)
    d = np.abs(np.diag(R))
    r = int(np.sum(d > tol))
    return Q[:, :r]


def eigh_desc(T: np.ndarray):
    """Symmetric eigendecomposition, eigenvalues in descending order."""
    w, V = np.linalg.eigh(0.5 * (T + T.T))
    return w[::-1], V[:, ::-1]


# ----------------------------------------------------------------------------- the Z operator

class ZOperator:
    """Z = X~ - alpha * grad f(X~) with X~ = W H^T and grad f(X~) = R on Omega
    (eq. zt), applied to thin matrices without forming Z:
        Z B   = W (H^T B) - alpha * (R B)        (B: n x q)
        Z^T U = H (W^T U) - alpha * (R^T U)      (U: m x q)."""

    def __init__(self, prob, W, H, R, alpha):
        self.prob, self.W, self.H, self.R, self.alpha = prob, W, H, R, alpha

    def matmul(self, B):
        out = -self.alpha * spmm(self.prob, self.R, B)
        if self.W.shape[1]:
            out += self.W @ (self.H.T @ B)
        return out

    def rmatmul(self, U):
        out = -self.alpha * spmm_t(self.prob, self.R, U)
        if self.W.shape[1]:
            out += self.H @ (self.W.T @ U)
        return out

    def fro2(self) -> float:
        """||Z||_F^2 = ||X~||^2 - 2 alpha <X~, R> + alpha^2 ||R||^2 (factored form)."""
        x2 = fro2_factored(self.W, self.H)
        xr = float(np.dot(self.R + self.prob.val, self.R)) if self.prob.nnz else 0.0
        return x2 - 2.0 * self.alpha * xr + self.alpha ** 2 * float(np.dot(self.R, self.R))


def fro2_factored(W, H) -> float:
    """||W H^T||_F^2 = tr((W^T W)(H^T H))."""
    if W.shape[1] == 0:
        return 0.0
    return float(np.sum((W.T @ W) * (H.T @ H)))


def diff_fro2_factored(W1, H1, W0, H0) -> float:
    """||W1 H1^T - W0 H0^T||_F^2 by eq. trace (Suppl. B.1) with the cross term
    carrying its factor -2:
        tr(W1'W1 H1'H1) + tr(W0'W0 H0'H0) - 2 tr((W0'W1)(H1'H0))."""
    a = fro2_factored(W1, H1)
    b = fro2_factored(W0, H0)
    if W1.shape[1] == 0 or W0.shape[1] == 0:
        return max(a + b, 0.0)
    c = float(np.sum((W0.T @ W1) * (H0.T @ H1)))
    return max(a + b - 2.0 * c, 0.0)


# ----------------------------------------------------------------------------- approximate SVD

@dataclass
class LmsvdResult:
    Uhat: np.ndarray      # m x q' orthonormal (columns with s > eps)
    Y: np.ndarray         # Z^T Uhat (n x q')
    iters: int
    ritz: np.ndarray      # eigenvalues of L^{t,i} at the last iteration


SSI_EPS = 1e-12          # Algorithm 2's cut of small s, relative to the largest
LMSVD_EIG_TOL = 1e-6     # cut of the small eigenvalues of P^T P (eq. PUi; history columns
                         # have unit norm, so the eigenvalues lie in [0, p])


def lmsvd(zop: ZOperator, U0: np.ndarray, tau: float, max_iter: int = 50,
          keep_level: float = 0.0, p: int = 0, trace: Optional[list] = None) -> LmsvdResult:
    """Algorithm 2 (LmSVD) with history length p_t = p (Suppl. A.1.2).

    L_t(U) = Z Z^T U.  The block subspace S_{t,i} is ran(U^{t,i}, ..., U^{t,i-p'})
    with p' = min(p, i) and U^{t,j} = orth(L_t(Uhat^{t,j-1})).  Its orthonormal
    basis is Q = [U^{t,i}, P S] (eq. orth-W): P projects the history blocks onto
    ker((U^{t,i})^T) (eq. PUi) and S = U~ Lambda^{-1/2} over the eigenpairs of
    P^T P above LMSVD_EIG_TOL (the trimming of nearly zero eigenvalues).  The
    subspace optimisation (eq. lmsvd-opt) keeps the k_t leading eigenvectors V of
    L^{t,i} = Q^T L_t(Q) = (Z^T Q)^T (Z^T Q); Uhat^{t,i} = Q V, and
    U^{t,i+1} = orth(L_t(Uhat^{t,i})).  Z^T Q needs no new product:
    Z^T P = Z^T U_old - (Z^T U^{t,i}) C with C = (U^{t,i})^T U_old.
    With p = 0, Q = U^{t,i} and this is the block subspace iteration with a
    Rayleigh-Ritz rotation.
    The loop stops once the k_t leading eigenvalues of L^{t,i} above
    ``keep_level`` (those the threshold will keep: the square of alpha * lambda)
    differ from those of L^{t,i-1} by at most tau * (largest eigenvalue).
    Output columns are those of the last U with s_j = ||Z^T u_j|| > eps.
    ``trace``, when given, receives per iteration the basis Q, the history block
    U_old, the eigenvalues of P^T P and the k_t leading Ritz values."""
    U = orth(U0)
    Y = zop.rmatmul(U)
    hist = []                      # (U^{t,j}, Z^T U^{t,j}) for j = i-1, ..., i-p'
    prev = None
    it = 0
    theta = np.zeros(0)
    for it in range(1, max_iter + 1):
        kt = U.shape[1]
        Q, Qz, lam, Uold = U, Y, np.zeros(0), None
        if hist:
            Uold = np.column_stack([h[0] for h in hist])
            Yold = np.column_stack([h[1] for h in hist])
            C = U.T @ Uold
            Pm = Uold - U @ C                                  # eq. PUi
            lam, Ut = eigh_desc(Pm.T @ Pm)
            keep = lam > LMSVD_EIG_TOL
            S = Ut[:, keep] / np.sqrt(lam[keep])
            Q = np.column_stack([U, Pm @ S])                   # eq. orth-W
            Qz = np.column_stack([Y, (Yold - Y @ C) @ S])      # Z^T Q
        th, V = eigh_desc(Qz.T @ Qz)                           # L^{t,i}
        theta, V = th[:kt], V[:, :kt]                          # eq. lmsvd-opt
        if trace is not None:
            trace.append({"Q": Q, "Uold": Uold, "lam": lam, "theta": theta})
        Unew = orth(zop.matmul(Qz @ V))                        # orth(L_t(Q V))
        if p > 0:
            hist = ([(U, Y)] + hist)[:p]
        U = Unew
        Y = zop.rmatmul(U)
        done = False
        if prev is not None and len(prev) == len(theta) and len(theta) > 0:
            J = theta > keep_level
            J[0] = True
            done = float(np.max(np.abs(theta[J] - prev[J]))) <= tau * max(theta[0], 0.0)
        prev = theta
        if done or U.shape[1] == 0:
            break
    s = np.linalg.norm(Y, axis=0)
    J = s > SSI_EPS * (s.max() if s.size else 0.0)
    return LmsvdResult(U[:, J], Y[:, J], it, theta)


@dataclass
class ProxResult:
    W: np.ndarray
    H: np.ndarray
    U: np.ndarray          # left singular vectors of Z~ (all q', sorted by sigma_hat)
    sigma_hat: np.ndarray  # singular values of Uhat^T Z
    sigma: np.ndarray      # thresholded, nonzero only
    k: int                 # new rank


def prox_from_basis(Uhat: np.ndarray, Y: np.ndarray, beta: float) -> ProxResult:
    """Exact SVD of Uhat^T Z (= Y^T) and singular-value soft-thresholding
    (eqs. exactSVD, approxSVD, truncate; Suppl. A.1.1):
        Uhat^T Z = U~ diag(sigma_hat) V^T,  U = Uhat U~,  Sigma = [sigma_hat - beta]_+ ,
    only strictly positive entries kept; W = U sqrt(Sigma), H = V sqrt(Sigma)
    (Algorithm 1, the W/H update)."""
    m, n = Uhat.shape[0], Y.shape[0]
    if Uhat.shape[1] == 0:
        return ProxResult(np.zeros((m, 0)), np.zeros((n, 0)), np.zeros((m, 0)), np.zeros(0),
                          np.zeros(0), 0)
    B = Y.T                                   # q' x n
    Ut, sig_hat, Vt = np.linalg.svd(B, full_matrices=False)
    U = Uhat @ Ut
    V = Vt.T
    sig = sig_hat - beta
    k = int(np.sum(sig > 0))
    sq = np.sqrt(sig[:k])
    return ProxResult(U[:, :k] * sq, V[:, :k] * sq, U, sig_hat, sig[:k], k)


# ----------------------------------------------------------------------------- safeguard (Suppl. A.1.3)

def safeguard_column(Ubase: np.ndarray, u: Optional[np.ndarray], psi: float, seed: int, t: int):
    """The extra column u_t + xi_t of eq. rt.

    u_t is the retained vector u projected onto ker(Ubase^T) (zero if there is
    none).  xi_t is a standard normal vector (stream STREAM_SAFEGUARD + t)
    projected onto ker([Ubase, u_t]^T) and scaled to norm psi.  With no retained
    vector the column is a unit random vector orthogonal to Ubase."""
    m = Ubase.shape[0]
    z = rng.normals(seed, rng.STREAM_SAFEGUARD + t, m)
    basis = Ubase
    ut = np.zeros(m)
    if u is not None:
        ut = u - Ubase @ (Ubase.T @ u) if Ubase.shape[1] else u.copy()
        nu = np.linalg.norm(ut)
        if nu > 0:
            basis = np.column_stack([Ubase, ut / nu])
    if basis.shape[1]:
        z = z - basis @ (basis.T @ z)
    nz = np.linalg.norm(z)
    xi = z / nz if nz > 0 else z
    if u is None:
        return xi
    return ut + psi * xi


# ----------------------------------------------------------------------------- initialisation (Suppl. A.1.4)

def pinv_psd(C: np.ndarray, rel: float = 1e-12) -> np.ndarray:
    """Pseudo-inverse of a symmetric PSD matrix, eigenvalues below rel * max as 0."""
    w, V = eigh_desc(C)
    if w.size == 0 or w[0] <= 0:
        return np.zeros_like(C)
    inv = np.where(w > rel * w[0], 1.0 / np.where(w > 0, w, 1.0), 0.0)
    return (V * inv) @ V.T


def initialize(prob, lam: float, k0: int, seed: int):
    """X_{-1} = 0 and one inexact PG step with alpha_{-1} = 1/L = 1:
    Z_{-1} = -grad f(0) = P_Omega(A).  A_{-1} = Z Z^T is approximated by the HMT
    range finder + Nystrom (eq. nys): Q = orth(A_{-1} Om), AQ = A_{-1} Q,
    C = Q^T AQ, AQ = Q^ R^ (QR), eig(R^ C^+ R^^T) = U~ diag(sigma^2) U~^T,
    Uhat_0 = Q^ U~ (positive eigenvalues only); then the exact-SVD / threshold
    tail of Suppl. A.1.1 with beta = lambda."""
    m, n = prob.m, prob.n
    zop = ZOperator(prob, np.zeros((m, 0)), np.zeros((n, 0)), -prob.val, 1.0)
    Om = rng.normals(seed, rng.STREAM_SKETCH, m * k0).reshape(m, k0)
    Q = orth(zop.matmul(zop.rmatmul(Om)))
    if Q.shape[1] == 0:
        z = np.zeros((m, 0))
        return ProxResult(z, np.zeros((n, 0)), z, np.zeros(0), np.zeros(0), 0), zop
    AQ = zop.matmul(zop.rmatmul(Q))
    C = Q.T @ AQ
    Qh, Rh = np.linalg.qr(AQ)
    M = Rh @ pinv_psd(C) @ Rh.T
    w, Ut = eigh_desc(M)
    pos = w > SSI_EPS * max(w[0], 0.0) if w.size else np.zeros(0, bool)
    Uhat0 = Qh @ Ut[:, pos]
    Y = zop.rmatmul(Uhat0)
    return prox_from_basis(Uhat0, Y, lam * 1.0), zop


# ----------------------------------------------------------------------------- the solver

@dataclass
class Options:
    lam: float
    k0: int
    alpha: float = 1.99          # fixed PG step for MC (Sec. 6.1: L = 1, alpha = 1.99)
    tol: float = 1e-6            # relative optimality residual
    bm_epochs: int = 3           # y (Sec. 6.1.1)
    max_iter: int = 500
    ssi_max_iter: int = 50
    ssi_tol_floor: float = 1e-12
    psi0: float = 0.1
    seed: int = 0
    lmsvd_p: int = 0             # p_t of Algorithm 2 (history blocks)
    # PG step size: "fixed" (alpha every step) or "sparsa" (Suppl. on the SpaRSA
    # variant: BB step of eq. proxBB clipped to [alpha_min, alpha_max], then
    # backtracking by sparsa_beta until eq. back holds with sparsa_delta)
    step_rule: str = "fixed"
    bm_solver: str = "polymf"    # "polymf": polyMF-SS (the paper's); "psd": preconditioned steepest descent
    alpha_min: float = 1.99      # < 2 delta / L (L = 1): eq. back holds there
    alpha_max: float = 1e3
    sparsa_beta: float = 0.5
    sparsa_delta: float = 0.999


@dataclass
class IterRecord:
    t: int
    F: float
    F_bm: float
    residual: float
    k: int
    q: int
    ssi_iters: int
    eps: float
    added_column: bool
    alpha: float = 1.99          # step of the accepted PG step
    trials: int = 1              # prox computations of the step (backtracking)


@dataclass
class SolveResult:
    W: np.ndarray
    H: np.ndarray
    k: int
    F: float
    residual: float
    iters: int
    converged: bool
    history: List[IterRecord] = field(default_factory=list)


def prox_step_standalone(prob, W, H, lam: float, alpha: float = 1.99, seed: int = 0,
                         tau: float = 1e-12, max_iter: int = 50, p: int = 0):
    """One inexact PG step from X~ = W H^T with no history: warm start orth(W~)
    (eq. rt0 without a previous prox output) plus the safeguard column of eq. rt
    with no retained vector (a unit random vector, stream STREAM_SAFEGUARD + 0),
    Algorithm 2 with history length p to tolerance tau, exact SVD and threshold
    alpha*lam.
    Returns (ProxResult, LmsvdResult, relative residual).  For m > n the step
    runs on the transpose (Sec. 1) and the output factors are swapped back."""
    if prob.m > prob.n:
        pr, ls, res = prox_step_standalone(transpose(prob), H, W, lam, alpha, seed, tau, max_iter, p)
        pr.W, pr.H = pr.H, pr.W
        return pr, ls, res
    R = sddmm(prob, W, H)
    zop = ZOperator(prob, W, H, R, alpha)
    Ubase = orth(W)
    U0 = orth(np.column_stack([Ubase, safeguard_column(Ubase, None, 0.0, seed, 0)]))
    ls = lmsvd(zop, U0, tau, max_iter, (alpha * lam) ** 2, p)
    pr = prox_from_basis(ls.Uhat, ls.Y, alpha * lam)
    return pr, ls, relative_residual(prob, W, H, R, ls.Uhat, pr.W, pr.H)


def ssi_tolerance(res_prev: float, floor: float) -> float:
    """tau_t = max(floor, min(1e-4, 0.1 res_{t-1}^2)): tightens with the outer
    residual so the prox errors eps_t are square-summable (Thm. conv)."""
    return max(floor, min(1e-4, 0.1 * res_prev * res_prev))


def step_norm(Uhat: np.ndarray, Wt, Ht, Wn, Hn) -> float:
    """||X~ - X+||_F where X+ = Wn Hn^T has its column space inside ran(Uhat)
    (true for the output of prox_from_basis).  With P = Uhat Uhat^T,
        ||X~ - X+||^2 = ||Uhat^T X~ - Uhat^T X+||^2 + ||(I - P) X~||^2,
    the first term from an explicit q x n difference, the second from
    E = W~ - Uhat (Uhat^T W~) as tr((E^T E)(H~^T H~)).  Unlike the three-trace
    identity (eq. trace) this has no cancellation between large terms, so it
    resolves steps far below 1e-8 * ||X||."""
    if Uhat.shape[1] == 0:
        return float(np.sqrt(fro2_factored(Wt, Ht) + fro2_factored(Wn, Hn)))
    D = (Uhat.T @ Wt) @ Ht.T
    if Wn.shape[1]:
        D = D - (Uhat.T @ Wn) @ Hn.T
    E = Wt - Uhat @ (Uhat.T @ Wt)
    out = float(np.sum(D * D))
    if Wt.shape[1]:
        out += float(np.sum((E.T @ E) * (Ht.T @ Ht)))
    return float(np.sqrt(out))


def relative_residual(prob, Wt, Ht, R, Uhat, Wn, Hn) -> float:
    """||X~ - X+||_F / (1 + ||X~||_F + ||grad f(X~)||_F) with X+ the PG output
    (the prox-gradient residual at step alpha scaled by alpha, which bounds the
    one at alpha = 1 from above)."""
    d = step_norm(Uhat, Wt, Ht, Wn, Hn)
    return d / (1.0 + np.sqrt(fro2_factored(Wt, Ht)) + np.sqrt(sumsq(prob, R)))


def diff_fro2_split(W1, H1, W0, H0) -> float:
    """||W1 H1^T - W0 H0^T||_F^2 for two nearby iterates.  eq. trace adds three
    traces of size ||X||^2 and loses all digits once the difference is below
    ~1e-8 ||X||.  With Q an orthonormal basis of ran(W1) and E_i = (I - Q Q^T) W_i,
        ||dX||^2 = ||(Q^T W1) H1^T - (Q^T W0) H0^T||_F^2 + ||E1 H1^T - E0 H0^T||_F^2
    (Pythagoras over ran(Q) and its complement): the first term is an explicit
    difference, the second eq. trace on the small remainders E_i."""
    if W1.shape[1] == 0 or W0.shape[1] == 0:
        return diff_fro2_factored(W1, H1, W0, H0)
    Q = orth(W1)
    D = (Q.T @ W1) @ H1.T - (Q.T @ W0) @ H0.T
    E1 = W1 - Q @ (Q.T @ W1)
    E0 = W0 - Q @ (Q.T @ W0)
    return float(np.sum(D * D)) + diff_fro2_factored(E1, H1, E0, H0)


def bb_step(W, H, Wp, Hp, R, Rp, alpha_min: float, alpha_max: float) -> float:
    """Barzilai-Borwein step of eq. proxBB between the PG points X~_t = W H^T and
    X~_{t-1} = Wp Hp^T, with R, Rp the sampled residuals there (grad f = R on
    Omega), read as the step
        ||X~_t - X~_{t-1}||_F^2 / <X~_t - X~_{t-1}, grad f(X~_t) - grad f(X~_{t-1})>,
    the numerator by diff_fro2_split (eq. trace rearranged so that nothing
    cancels) and the denominator ||R - Rp||^2 since
    grad f(X) - grad f(Y) = P_Omega(X - Y) for (MC); clipped to
    [alpha_min, alpha_max] (alpha_max when the denominator vanishes)."""
    num = diff_fro2_split(W, H, Wp, Hp)
    den = float(np.dot(R - Rp, R - Rp))
    a = num / den if den > 0.0 else alpha_max
    return min(alpha_max, max(alpha_min, a))


def back_condition(prob, R, Wn, Hn, d2: float, alpha: float, delta: float):
    """eq. back at X+ = Wn Hn^T from X~ with sampled residual R:
        f(X+) <= f(X~) + <grad f(X~), X+ - X~> + delta / alpha ||X+ - X~||^2,
    d2 = ||X+ - X~||_F^2.  The MC loss is quadratic, so
        f(X+) - f(X~) - <grad f(X~), X+ - X~> = 1/2 ||P_Omega(X+ - X~)||^2
                                              = 1/2 ||R+ - R||^2
    exactly (R+ the residual at X+), and the test is made in that form: the
    three f terms are large and nearly cancel once steps are small.  Returns
    (holds, left side 1/2 ||R+ - R||^2, right side delta / alpha * d2)."""
    Rn = sddmm(prob, Wn, Hn)
    lhs = 0.5 * float(np.dot(Rn - R, Rn - R))
    rhs = delta / alpha * d2
    return lhs <= rhs, lhs, rhs


def solve(prob, opt: Options, callback=None) -> SolveResult:
    """Runs :func:`_solve` with single-threaded BLAS (the dense steps are small;
    threaded BLAS only adds contention with the OpenMP sparse loops).  The
    method assumes m <= n (Sec. 1: otherwise transpose), so a problem with
    m > n is solved as its transpose and the factors are swapped back."""
    with threadpool_limits(limits=1, user_api="blas"):
        if prob.m > prob.n:
            res = _solve(transpose(prob), opt, callback)
            res.W, res.H = res.H, res.W
            return res
        return _solve(prob, opt, callback)


def _solve(prob, opt: Options, callback=None) -> SolveResult:
    """Algorithm 1 (BM-Global) for (MC): per outer iteration y BM epochs, then
    one inexact PG step with warm start (eqs. rt0 / rt0-1), rank safeguard
    (eq. rt), LmSVD (Algorithm 2), exact SVD + threshold, and the rank
    update k = rank(Sigma).  With step_rule "sparsa" the step from the second
    PG step on is the BB step (bb_step) times sparsa_beta^i for the smallest i
    whose prox output satisfies eq. back, floored at alpha_min (where eq. back
    holds for L = 1); every trial restarts LmSVD from the same warm start.  The
    stopping residual is ||X~ - X+|| at the accepted alpha_t unscaled: it does
    not decrease with the step (alpha ||G_alpha|| is nondecreasing in alpha for
    the prox-gradient mapping G_alpha), so for alpha_t >= alpha it bounds the
    fixed-step residual from above."""
    sparsa = opt.step_rule == "sparsa"
    if opt.step_rule not in ("fixed", "sparsa"):
        raise ValueError("step_rule must be 'fixed' or 'sparsa'")
    if opt.bm_solver not in ("psd", "polymf"):
        raise ValueError("bm_solver must be 'psd' or 'polymf'")
    prev_pt = None                                  # (W~, H~, R) of the previous PG step
    lam, alpha = opt.lam, opt.alpha
    init, _ = initialize(prob, lam, opt.k0, opt.seed)
    W, H = init.W, init.H
    U_cur = init.U[:, :init.k]                      # left singular vectors of X_0
    U_prev = np.zeros((prob.m, 0))                  # of X_{-1} = 0
    rank_cur, rank_prev = init.k, 0
    trunc_prev = len(init.sigma_hat) - init.k       # truncated at the previous PG step
    u_keep = init.U[:, init.k].copy() if trunc_prev >= 1 else None
    psi = opt.psi0
    res_prev = 1.0
    hist: List[IterRecord] = []
    F = objective(prob, W, H, lam)
    res = np.inf
    converged = False
    t = 0
    for t in range(opt.max_iter):
        # ---- BM phase (y epochs)
        Wt, Ht = W, H
        for _ in range(opt.bm_epochs):
            if Wt.shape[1] == 0:
                break
            if opt.bm_solver == "polymf":
                Wt, Ht, _ = polymf_epoch(prob, Wt, Ht, lam)
            else:
                Wt, Ht, _ = bm_epoch(prob, Wt, Ht, lam)
        F_bm = bm_objective(prob, Wt, Ht, lam)
        changed = not (np.array_equal(Wt, W) and np.array_equal(Ht, H))
        # ---- convex lifting: Z_t = X~_t - alpha grad f(X~_t)
        R = sddmm(prob, Wt, Ht)
        Ubase = orth(np.column_stack([U_cur, Wt if changed else U_prev]))
        add = trunc_prev <= 1 or rank_cur == rank_prev or Ubase.shape[1] == 0
        if add:
            U0 = orth(np.column_stack([Ubase, safeguard_column(Ubase, u_keep, psi, opt.seed, t)]))
        else:
            U0 = Ubase
        tau = ssi_tolerance(res_prev, opt.ssi_tol_floor)
        a = alpha
        if sparsa and prev_pt is not None:
            a = bb_step(Wt, Ht, prev_pt[0], prev_pt[1], R, prev_pt[2], opt.alpha_min, opt.alpha_max)
        trials, ssi_sum = 0, 0
        while True:
            trials += 1
            zop = ZOperator(prob, Wt, Ht, R, a)
            ls = lmsvd(zop, U0, tau, opt.ssi_max_iter, (a * lam) ** 2, opt.lmsvd_p)
            ssi_sum += ls.iters
            pr = prox_from_basis(ls.Uhat, ls.Y, a * lam)
            if not sparsa or a <= opt.alpha_min:
                break
            d = step_norm(ls.Uhat, Wt, Ht, pr.W, pr.H)
            if back_condition(prob, R, pr.W, pr.H, d * d, a, opt.sparsa_delta)[0]:
                break
            a = max(opt.alpha_min, a * opt.sparsa_beta)
        if sparsa:
            prev_pt = (Wt, Ht, R)
        eps2 = zop.fro2() - float(np.sum(pr.sigma_hat ** 2))
        res = relative_residual(prob, Wt, Ht, R, ls.Uhat, pr.W, pr.H)
        # ---- safeguard bookkeeping
        q = len(pr.sigma_hat)
        trunc = q - pr.k
        if trunc >= 1:
            u_keep = pr.U[:, pr.k].copy()
        else:
            u_keep = None
        if trunc == 1:
            psi *= 0.5
        trunc_prev = trunc
        U_prev, U_cur = U_cur, pr.U[:, :pr.k]
        rank_prev, rank_cur = rank_cur, pr.k
        W, H = pr.W, pr.H
        F = objective(prob, W, H, lam)
        rec = IterRecord(t, F, F_bm, res, pr.k, q, ssi_sum, float(np.sqrt(max(eps2, 0.0))), add,
                         a, trials)
        hist.append(rec)
        if callback:
            callback(rec)
        res_prev = res
        if res <= opt.tol:
            converged = True
            break
    return SolveResult(W, H, W.shape[1], F, res, t + 1, converged, hist)
