"""Pins of the kernel-estimation QSDP oracle (oracle/rke.py) against dense
definitions and independent routes (CPU only)."""
import math

import numpy as np
import pytest

import synth
from oracle import rke


def rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def dense_parts(p):
    rows, cols = p.rows(), p.col
    return rows, cols


def dense_lap(p, r):
    """A^*(r) as a dense n x n matrix: sum over stored (i, j) of r (e_i e_i^T - e_i e_j^T)."""
    rows, cols = dense_parts(p)
    L = np.zeros((p.n, p.n))
    np.add.at(L, (rows, rows), r)
    np.add.at(L, (rows, cols), -r)
    return L


def dense_f(p, X, lam):
    rows, cols = dense_parts(p)
    r = X[rows, rows] + X[cols, cols] - 2 * X[rows, cols] - p.val
    return 0.25 * float(r @ r) + lam * float(np.trace(X)), r


def test_pair_residual_and_laplacian_match_dense():
    p = synth.rke(30, 8, seed=4)
    W = rand((30, 3), 1)
    X = W @ W.T
    _, rd = dense_f(p, X, 0.0)
    r = rke.pair_residual(p, W)
    assert np.allclose(r, rd, atol=1e-12)
    U = rand((30, 5), 2)
    assert np.allclose(rke.lap_apply(p, r, U), dense_lap(p, r) @ U, atol=1e-11)
    # the Laplacian annihilates e and is symmetric
    L = dense_lap(p, r)
    assert np.allclose(L, L.T) and np.allclose(L @ np.ones(30), 0.0, atol=1e-12)


def test_bm_gradient_and_exact_quartic_step():
    p = synth.rke(30, 8, seed=5)
    lam = 0.7
    W = rke.center(rand((30, 3), 3))
    F = lambda V: rke.bm_objective(p, V, lam)  # noqa: E731
    # F~ = f(W W^T) + lam tr(W W^T) and its gradient 2 (L_r W + lam W)
    assert math.isclose(F(W), dense_f(p, W @ W.T, lam)[0], rel_tol=1e-12)
    r = rke.pair_residual(p, W)
    G = 2 * (rke.lap_apply(p, r, W) + lam * W)
    V = rand((30, 3), 6)
    h = 1e-6
    fd = (F(W + h * V) - F(W - h * V)) / (2 * h)
    assert math.isclose(fd, float(np.sum(G * V)), rel_tol=1e-6)
    # the line search is the exact minimiser along D
    D = -rke.center(G / 2)
    t = rke.quartic_step(p, W, D, r, lam)
    grid = np.linspace(0.0, 3.0 * t + 1e-3, 3001)
    vals = np.array([F(W + s * D) for s in grid])
    assert t > 0 and F(W + t * D) <= vals.min() + 1e-12 * abs(vals.min())


def test_bm_phase_is_monotone_and_keeps_the_constraint():
    p = synth.rke(40, 10, seed=6)
    W = rke.center(rand((40, 4), 7))
    Fs = [rke.bm_objective(p, W, 0.5)]
    for _ in range(4):
        W, ts = rke.bm_phase(p, W, 0.5, 3)
        Fs.append(rke.bm_objective(p, W, 0.5))
        assert all(t >= 0 for t in ts)
    assert all(b <= a * (1 + 1e-14) for a, b in zip(Fs, Fs[1:])) and Fs[-1] < Fs[0]
    assert np.allclose(W.sum(axis=0), 0.0, atol=1e-10)


def test_lemma_pix_against_reduced_coordinates():
    # {X psd, <E, X> = 0} = {Q Y Q^T : Y psd} with Q an orthonormal basis of the
    # complement of e (a psd X with e^T X e = 0 has X e = 0), and
    # ||Q Y Q^T - G||^2 = ||Y - Q^T G Q||^2 + const, so the projection is
    # Q P_S+(Q^T G Q) Q^T: a route that does not use the lemma
    for n, seed in ((8, 9), (15, 12)):
        A = rand((n, n), seed)
        G = A + A.T
        Q = np.linalg.svd(np.eye(n) - np.ones((n, n)) / n)[0][:, :n - 1]
        w, V = np.linalg.eigh(Q.T @ G @ Q)
        Xr = Q @ ((V * np.maximum(w, 0)) @ V.T) @ Q.T
        Pl = rke.project_dense(G)
        assert np.allclose(Pl, Xr, atol=1e-11)
        assert abs(np.sum(Pl)) < 1e-10 and np.linalg.eigvalsh(Pl).min() > -1e-10


@pytest.mark.parametrize("hist", [0, 1, 2])
def test_eig_prox_is_the_projection_of_the_pg_point(hist):
    """With and without the history of Algorithm 2: the same projection."""
    p = synth.rke(30, 10, seed=8)
    lam, alpha = 0.8, 1.99 / rke.lipschitz_bound(p)
    W = rke.center(rand((30, 3), 10))
    r = rke.pair_residual(p, W)
    Z = W @ W.T - alpha * (dense_lap(p, r) + lam * np.eye(30))
    Xd = rke.project_dense(Z)
    kd = int(np.sum(np.linalg.eigvalsh(Xd) > 1e-9))
    ep = rke.eig_prox(p, W, r, alpha, lam, rand((30, kd + 6), 11), 1e-14, max_iter=3000, p=hist)
    assert np.allclose(ep.W @ ep.W.T, Xd, atol=1e-8)
    assert ep.W.shape[1] == kd
    assert np.allclose(ep.W.sum(axis=0), 0.0, atol=1e-10)


@pytest.mark.parametrize("hist", [0, 1])
def test_solve_matches_dense_proximal_gradient(hist):
    p = synth.rke(50, 30, lam=2.0, seed=3)
    lam = 2.0
    res = rke.solve(p, lam, k0=6, tol=1e-8, seed=1, max_iter=1000, lmsvd_p=hist)
    alpha = 1.99 / rke.lipschitz_bound(p)
    X = np.zeros((p.n, p.n))
    for _ in range(100000):
        _, r = dense_f(p, X, lam)
        Xn = rke.project_dense(X - alpha * (dense_lap(p, r) + lam * np.eye(p.n)))
        if np.linalg.norm(Xn - X) < 1e-12 * (1 + np.linalg.norm(X)):
            X = Xn
            break
        X = Xn
    Fd = dense_f(p, X, lam)[0]
    assert res.converged
    assert math.isclose(res.F, Fd, rel_tol=1e-10)
    assert res.k == np.linalg.matrix_rank(X, tol=1e-7)
    assert np.allclose(res.W.sum(axis=0), 0.0, atol=1e-9)
