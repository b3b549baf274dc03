"""The library's small host FP64 linear algebra (csrc/linalg.cpp) against its
definitions, on the CPU.  The source is compiled here with g++ twice, as the
library builds it (baseline x86-64 and x86-64-v3), behind a C shim of this
test's own; numpy supplies the reference decompositions."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                    "paper_2204_14067_amd", "csrc")

SHIM = r"""
namespace bmg { namespace la_t {
void sym_eig(int n, const double *A, double *w, double *V);
int chol_pivoted(int n, const double *G, double tol, int *perm, double *R);
bool chol(int n, const double *G, double *R);
void tri_inv_upper(int n, const double *R, double *Rinv);
bool spd_inv(int n, const double *A, double *Ainv);
} }
extern "C" {
void t_sym_eig(int n, const double *A, double *w, double *V) { bmg::la_t::sym_eig(n, A, w, V); }
int t_chol_pivoted(int n, const double *G, double tol, int *perm, double *R) {
  return bmg::la_t::chol_pivoted(n, G, tol, perm, R);
}
int t_chol(int n, const double *G, double *R) { return bmg::la_t::chol(n, G, R); }
void t_tri_inv_upper(int n, const double *R, double *X) { bmg::la_t::tri_inv_upper(n, R, X); }
int t_spd_inv(int n, const double *A, double *X) { return bmg::la_t::spd_inv(n, A, X); }
}
"""

FLAGS = {"generic": [], "v3": ["-march=x86-64-v3"]}


def _cpu_has_v3():
    try:
        with open("/proc/cpuinfo") as f:
            flags = f.read()
        return " avx2" in flags and " fma" in flags
    except OSError:
        return False


@pytest.fixture(scope="module", params=sorted(FLAGS))
def la(request, tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    if request.param == "v3" and not _cpu_has_v3():
        pytest.skip("host CPU lacks AVX2/FMA")
    d = tmp_path_factory.mktemp("la_" + request.param)
    shim = d / "shim.cpp"
    shim.write_text(SHIM)
    so = d / "libla_t.so"
    subprocess.run(["g++", "-O3", "-fPIC", "-shared", "-DLA_IMPL=la_t", *FLAGS[request.param],
                    os.path.join(CSRC, "linalg.cpp"), str(shim), "-o", str(so)], check=True)
    lib = ctypes.CDLL(str(so))
    P = ctypes.POINTER(ctypes.c_double)
    lib.t_sym_eig.argtypes = [ctypes.c_int, P, P, P]
    lib.t_chol_pivoted.argtypes = [ctypes.c_int, P, ctypes.c_double, ctypes.POINTER(ctypes.c_int), P]
    lib.t_chol.argtypes = [ctypes.c_int, P, P]
    lib.t_tri_inv_upper.argtypes = [ctypes.c_int, P, P]
    lib.t_spd_inv.argtypes = [ctypes.c_int, P, P]
    return lib


def ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def sym_eig(lib, A, vectors=True):
    n = A.shape[0]
    A = np.ascontiguousarray(A, dtype=np.float64)
    w = np.zeros(n)
    V = np.zeros((n, n)) if vectors else None
    lib.t_sym_eig(n, ptr(A), ptr(w), ptr(V) if vectors else None)
    return w, V


def rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def eig_cases():
    out = []
    for n, seed in ((1, 1), (2, 2), (3, 3), (17, 4), (92, 5), (183, 6)):
        B = rand((n, n), seed)
        out.append(("gram%d" % n, B @ B.T))
        out.append(("indef%d" % n, B + B.T))
    B = rand((60, 10), 7)
    out.append(("rank10_of_60", B @ B.T))
    Q = np.linalg.qr(rand((40, 40), 8))[0]
    w = np.repeat([5.0, 2.0, 2.0 + 1e-13, -1.0, 0.0], 8)
    out.append(("clustered40", (Q * w) @ Q.T))
    out.append(("graded30", (Q[:30, :30] * np.logspace(0, -12, 30)) @ Q[:30, :30].T))
    out.append(("diag", np.diag([3.0, -1.0, 7.0, 0.0, 2.0])))
    out.append(("zero", np.zeros((6, 6))))
    out.append(("tridiag", np.diag(np.full(50, 2.0)) - np.diag(np.ones(49), 1) - np.diag(np.ones(49), -1)))
    return out


@pytest.mark.parametrize("name,A", eig_cases(), ids=[c[0] for c in eig_cases()])
def test_sym_eig_against_numpy(la, name, A):
    n = A.shape[0]
    w, V = sym_eig(la, A)
    scale = max(1.0, np.abs(A).max()) * n
    ref = np.sort(np.linalg.eigvalsh(A))[::-1]
    assert np.all(np.diff(w) <= 0.0), "eigenvalues not in descending order"
    assert np.allclose(w, ref, rtol=0, atol=1e-13 * scale)
    assert np.allclose(V.T @ V, np.eye(n), rtol=0, atol=1e-13 * n)
    assert np.allclose((V * w) @ V.T, A, rtol=0, atol=1e-13 * scale)
    # the values-only call runs the same tridiagonal iteration
    w0, _ = sym_eig(la, A, vectors=False)
    assert np.array_equal(w0, w)


def test_sym_eig_uses_the_mean_of_a_and_its_transpose(la):
    A = rand((9, 9), 11)
    w, V = sym_eig(la, A)
    S = 0.5 * (A + A.T)
    assert np.allclose((V * w) @ V.T, S, rtol=0, atol=1e-12)


def test_cholesky_triangular_inverse_and_spd_inverse(la):
    for n, seed in ((1, 1), (5, 2), (64, 3), (150, 4)):
        B = rand((n, n + 3), seed)
        G = B @ B.T
        R = np.zeros((n, n))
        assert la.t_chol(n, ptr(G), ptr(R))
        assert np.allclose(np.tril(R, -1), 0.0)
        assert np.all(np.diag(R) > 0)
        assert np.allclose(R.T @ R, G, rtol=0, atol=1e-12 * np.abs(G).max())
        X = np.zeros((n, n))
        la.t_tri_inv_upper(n, ptr(R), ptr(X))
        assert np.allclose(R @ X, np.eye(n), rtol=0, atol=1e-9)
        Gi = np.zeros((n, n))
        assert la.t_spd_inv(n, ptr(G), ptr(Gi))
        assert np.allclose(Gi, Gi.T, rtol=0, atol=0)
        assert np.allclose(G @ Gi, np.eye(n), rtol=0, atol=1e-8)
    # not positive definite
    B = rand((6, 3), 5)
    G = B @ B.T - 1e-3 * np.eye(6)
    R = np.zeros((6, 6))
    assert not la.t_chol(6, ptr(G), ptr(R))
    assert not la.t_spd_inv(6, ptr(G), ptr(R))


def test_pivoted_cholesky_finds_the_rank(la):
    n, r = 40, 7
    B = rand((n, r), 12) * np.logspace(0, -3, r)
    G = B @ B.T
    R = np.zeros((n, n))
    perm = np.zeros(n, dtype=np.int32)
    got = la.t_chol_pivoted(n, ptr(G), 1e-12, perm.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), ptr(R))
    assert got == r
    assert sorted(perm.tolist()) == list(range(n))
    Rr = R[:r]
    assert np.allclose(np.tril(Rr[:, :r], -1), 0.0)
    # the pivot takes the largest remaining diagonal, so |R_jj| is non-increasing
    d = np.abs(np.diag(Rr[:, :r]))
    assert np.all(np.diff(d) <= 1e-12 * d[0])
    Gp = G[np.ix_(perm, perm)]
    assert np.allclose(Rr.T @ Rr, Gp, rtol=0, atol=1e-12 * np.abs(G).max())
    # full rank with a zero tolerance; a zero matrix has rank 0
    G2 = rand((12, 12), 13)
    G2 = G2 @ G2.T
    R2 = np.zeros((12, 12))
    p2 = np.zeros(12, dtype=np.int32)
    assert la.t_chol_pivoted(12, ptr(G2), 0.0, p2.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), ptr(R2)) == 12
    Z = np.zeros((4, 4))
    assert la.t_chol_pivoted(4, ptr(Z), 1e-12, p2.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                             ptr(np.zeros((4, 4)))) == 0
