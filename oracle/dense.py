"""Small dense references that pin the oracle (FP64, CPU).

TEST INFRASTRUCTURE ONLY (see the package docstring).  These functions solve
the same mathematics by a different route (full SVDs of explicit matrices,
LAPACK/ARPACK), so a mistake in ``core`` shows up as a disagreement.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def to_dense(prob):
    """Explicit A (zeros off Omega) and the 0/1 mask of Omega."""
    A = np.zeros((prob.m, prob.n))
    M = np.zeros((prob.m, prob.n), bool)
    rows = prob.rows()
    A[rows, prob.col] = prob.val
    M[rows, prob.col] = True
    return A, M


def to_scipy(prob, vals=None):
    v = prob.val if vals is None else vals
    return sp.csr_matrix((v, prob.col, prob.row_ptr), shape=(prob.m, prob.n))


def prox_nuclear(Z: np.ndarray, beta: float) -> np.ndarray:
    """prox_{beta ||.||_*}(Z) = U diag([sigma - beta]_+) V^T (eq. proxnuc, Sec. 2)."""
    U, s, Vt = np.linalg.svd(Z, full_matrices=False)
    return (U * np.maximum(s - beta, 0.0)) @ Vt


def mc_objective_dense(X, A, M, lam) -> float:
    D = np.where(M, X - A, 0.0)
    return 0.5 * float(np.sum(D * D)) + lam * float(np.linalg.svd(X, compute_uv=False).sum())


def proximal_gradient_dense(A, M, lam, alpha=1.0, tol=1e-12, max_iter=100000, X0=None):
    """Exact PG for (MC) with full SVDs (soft-impute at alpha = 1, Sec. 5.1):
    X <- prox_{alpha lambda ||.||_*}(X - alpha P_Omega(X - A)) until
    ||X_new - X||_F <= tol * (1 + ||X||_F)."""
    X = np.zeros_like(A) if X0 is None else X0.copy()
    it = 0
    for it in range(1, max_iter + 1):
        Xn = prox_nuclear(X - alpha * np.where(M, X - A, 0.0), alpha * lam)
        d = np.linalg.norm(Xn - X)
        X = Xn
        if d <= tol * (1.0 + np.linalg.norm(X)):
            break
    return X, it


def spectral_norm(prob, vals) -> float:
    """||S||_2 of the sparse matrix with values ``vals`` on Omega (ARPACK, or a
    dense SVD up to 4,000 on the short side: at an optimum the top singular
    value of the gradient is lambda with the multiplicity of the rank, a
    cluster ARPACK may fail to converge on)."""
    if min(prob.m, prob.n) <= 4000:
        A, M = to_dense(prob)
        S = np.zeros((prob.m, prob.n))
        S[prob.rows(), prob.col] = vals
        return float(np.linalg.svd(S, compute_uv=False)[0])
    S = to_scipy(prob, vals)
    return float(spla.svds(S, k=1, return_singular_vectors=False, tol=1e-12)[0])


def duality_gap(prob, G_vals, F_primal: float, lam: float):
    """Fenchel dual of (MC): max over Lambda supported on Omega with
    ||Lambda||_2 <= lambda of  -1/2 ||Lambda||^2 - <Lambda, A>.  The gradient
    G = P_Omega(X - A) scaled into the feasible set gives a dual value D, and
    F(X) - F* <= F(X) - D.  Returns (gap, D, ||G||_2)."""
    g2 = spectral_norm(prob, G_vals)
    c = 1.0 if g2 <= lam else lam / g2
    L = c * G_vals
    D = -0.5 * float(np.dot(L, L)) - float(np.dot(L, prob.val))
    return F_primal - D, D, g2
