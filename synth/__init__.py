"""Seeded synthetic matrix-completion workloads.

Input generation only: this module draws the sampling pattern Omega and the
observed values A_Omega (and, for the serving stream, the request mix).  It
holds none of the solver's arithmetic; the CPU oracle and the GPU path both
read what it returns.

Workloads (all synthetic; no dataset records are reproduced):

* ``small_uniform``  1000 x 1500, |Omega| = 50,000 uniform without replacement,
  rank-5 Gaussian truth (factor entries of variance 1/sqrt(5), so the truth has
  unit-variance entries) plus noise of variance 0.01; lambda = 0.5, k0 = 8.
* ``netflix_shape``  17,770 x 480,189, |Omega| ~ 1e8, capped Zipf(1.2) row and
  column degrees, rank-20 truth plus noise of variance 0.25, ratings-like
  values 3 + truth + noise clipped to [1, 5]; lambda = 20, k0 = 16.
* ``yahoo_shape``    624,961 x 1,000,990, |Omega| ~ 2.5e8, capped power law
  (exponent 1.1), rank-30 truth plus noise of variance 0.5, unclipped;
  lambda = 50, k0 = 32.
* ``rke``            regularized kernel estimation: n objects in R^3, about
  deg/2 random partners each, noisy squared distances, symmetric storage.
* ``serving_stream`` 256 problems, Poisson arrivals at 20/s, m ~ U[500, 20000],
  n ~ U[1000, 50000], density ~ U[0.5%, 2%], rank ~ U{3..15}, noise variance
  0.05, lambda relative to the sampling/noise level (see serving_stream).

The ``scale`` argument shrinks a power-law workload (m, n and |Omega| by the
same factor) for tests that must finish in seconds on the oracle.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the generator (plain C, OpenMP) into synth/libsynth.so."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp,
                               os.path.join(_HERE, "gen.c"), "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        i64, p = ctypes.c_int64, ctypes.c_void_p
        lib.synth_uniform_pattern.argtypes = [i64, i64, i64, ctypes.c_uint64, p, p]
        lib.synth_uniform_pattern.restype = ctypes.c_int
        lib.synth_powerlaw_degrees.argtypes = [i64, i64, i64, ctypes.c_double, ctypes.c_uint64, p]
        lib.synth_powerlaw_degrees.restype = i64
        lib.synth_powerlaw_columns.argtypes = [i64, i64, ctypes.c_double, ctypes.c_uint64, p, p]
        lib.synth_powerlaw_columns.restype = ctypes.c_int
        lib.synth_values.argtypes = [i64, i64, p, p, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_uint64, p, p, p]
        lib.synth_values.restype = ctypes.c_int
        lib.synth_uniforms.argtypes = [ctypes.c_uint64, ctypes.c_uint64, i64, p]
        lib.synth_uniforms.restype = None
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Problem:
    """One completion problem: CSR of Omega with observed values, lambda, k0."""
    name: str
    m: int
    n: int
    row_ptr: np.ndarray          # int64 [m+1]
    col: np.ndarray              # int32 [nnz], sorted within each row
    val: np.ndarray              # float64 [nnz]
    lam: float
    k0: int
    U: Optional[np.ndarray] = None   # ground-truth factors (float64), if kept
    V: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def rows(self) -> np.ndarray:
        """Row index of every stored entry (int64 [nnz])."""
        return np.repeat(np.arange(self.m, dtype=np.int64), np.diff(self.row_ptr))


def uniform_pattern(m: int, n: int, nnz: int, seed: int):
    lib = _load()
    row_ptr = np.zeros(m + 1, np.int64)
    col = np.zeros(max(nnz, 1), np.int32)
    rc = lib.synth_uniform_pattern(m, n, nnz, seed, _ptr(row_ptr), _ptr(col))
    if rc != 0:
        raise ValueError("synth_uniform_pattern failed (%d)" % rc)
    return row_ptr, col[:nnz]


def powerlaw_pattern(m: int, n: int, N: int, a_row: float, a_col: float, seed: int):
    lib = _load()
    deg = np.zeros(m, np.int64)
    tot = lib.synth_powerlaw_degrees(m, n, N, a_row, seed, _ptr(deg))
    row_ptr = np.zeros(m + 1, np.int64)
    np.cumsum(deg, out=row_ptr[1:])
    assert row_ptr[-1] == tot
    col = np.zeros(max(tot, 1), np.int32)
    rc = lib.synth_powerlaw_columns(m, n, a_col, seed, _ptr(row_ptr), _ptr(col))
    if rc != 0:
        raise ValueError("synth_powerlaw_columns failed (%d)" % rc)
    return row_ptr, col[:tot]


def values(m, n, row_ptr, col, rank, var_f, var_e, offset=0.0, lo=1.0, hi=0.0, seed=0,
           keep_truth=False):
    lib = _load()
    nnz = int(row_ptr[-1])
    val = np.zeros(max(nnz, 1), np.float64)
    U = np.zeros((m, rank), np.float64) if keep_truth else None
    V = np.zeros((n, rank), np.float64) if keep_truth else None
    lib.synth_values(m, n, _ptr(row_ptr), _ptr(col), rank, var_f, var_e, offset, lo, hi, seed,
                     _ptr(val), _ptr(U), _ptr(V))
    return val[:nnz], U, V


def uniforms(seed: int, stream: int, count: int) -> np.ndarray:
    out = np.zeros(max(count, 1), np.float64)
    _load().synth_uniforms(seed, stream, count, _ptr(out))
    return out[:count]


# ----------------------------------------------------------------------------- workloads

def small_uniform(seed: int = 1001, m: int = 1000, n: int = 1500, nnz: int = 50_000, rank: int = 5,
                  var_e: float = 0.01, lam: float = 0.5, k0: int = 8, keep_truth=False) -> Problem:
    row_ptr, col = uniform_pattern(m, n, nnz, seed)
    val, U, V = values(m, n, row_ptr, col, rank, 1.0 / math.sqrt(rank), var_e, seed=seed + 7,
                       keep_truth=keep_truth)
    return Problem("small_uniform_%dx%d_nnz%d" % (m, n, nnz), m, n, row_ptr, col, val, lam, k0, U, V,
                   dict(seed=seed, rank=rank, var_e=var_e, pattern="uniform"))


def powerlaw(name: str, m: int, n: int, N: int, a: float, rank: int, var_e: float, offset: float,
             lo: float, hi: float, lam: float, k0: int, seed: int, scale: float = 1.0) -> Problem:
    if scale != 1.0:
        m, n, N = max(8, int(m * scale)), max(8, int(n * scale)), max(16, int(N * scale * scale))
    row_ptr, col = powerlaw_pattern(m, n, N, a, a, seed)
    val, _, _ = values(m, n, row_ptr, col, rank, 1.0 / math.sqrt(rank), var_e, offset, lo, hi,
                       seed=seed + 7)
    return Problem("%s_%dx%d_nnz%d" % (name, m, n, int(row_ptr[-1])), m, n, row_ptr, col, val, lam,
                   k0, meta=dict(seed=seed, rank=rank, var_e=var_e, exponent=a, pattern="powerlaw",
                                 scale=scale))


def netflix_shape(scale: float = 1.0, seed: int = 1002) -> Problem:
    return powerlaw("netflix_shape", 17_770, 480_189, 100_000_000, 1.2, 20, 0.25, 3.0, 1.0, 5.0,
                    20.0, 16, seed, scale)


def yahoo_shape(scale: float = 1.0, seed: int = 1003) -> Problem:
    return powerlaw("yahoo_shape", 624_961, 1_000_990, 250_000_000, 1.1, 30, 0.5, 0.0, 1.0, 0.0,
                    50.0, 32, seed, scale)


def movielens_shape(which: str = "100k", seed: int = 1007) -> Problem:
    """Rating-shaped stand-ins for the two small problems the paper times in
    its tables (Sec. 6.1): "100k" has the MovieLens-100k shape (943 x 1,682,
    90,570 entries, lambda 15), "toy" the toy example's (3,952 x 6,040,
    900,189 entries, lambda 36).  Power-law degrees (exponent 1.0 on rows and
    columns), values 3 + rank-10 Gaussian (factor variance 1/sqrt(10)) + noise
    of variance 0.25, clipped to [1, 5]; k0 = 8.  No record of either dataset
    is used: only their shapes and the paper's lambda."""
    if which == "100k":
        return powerlaw("movielens100k_shape", 943, 1_682, 90_570, 1.0, 10, 0.25, 3.0, 1.0, 5.0, 15.0, 8,
                        seed)
    if which == "toy":
        return powerlaw("toy_shape", 3_952, 6_040, 900_189, 1.0, 10, 0.25, 3.0, 1.0, 5.0, 36.0, 8, seed)
    raise ValueError("which must be '100k' or 'toy'")


def tiny(m: int, n: int, nnz: int, rank: int = 2, var_e: float = 0.01, lam: float = 0.1,
         k0: int = 4, seed: int = 7) -> Problem:
    """Small uniform problem for brute-force checks (nnz may be 0 or m*n)."""
    row_ptr, col = uniform_pattern(m, n, nnz, seed)
    val, U, V = values(m, n, row_ptr, col, rank, 1.0 / math.sqrt(rank), var_e, seed=seed + 7,
                       keep_truth=True)
    return Problem("tiny_%dx%d_nnz%d" % (m, n, nnz), m, n, row_ptr, col, val, lam, k0, U, V,
                   dict(seed=seed, rank=rank, var_e=var_e, pattern="uniform"))


def rke(n: int, deg: int, dim: int = 3, noise: float = 0.1, lam: float = 1.0, k0: int = 8,
        seed: int = 1006) -> Problem:
    """Regularized kernel estimation input (QSDP section): n objects at
    Gaussian positions in R^dim; each object draws deg/2 partners uniformly
    (pairs deduplicated), and each pair carries the squared distance times
    (1 + noise * N(0, 1)), floored at 0.  Stored as a symmetric n x n CSR with
    both (i, j) and (j, i) and the value d_ij^2."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, dim))
    half = max(1, deg // 2)
    i = np.repeat(np.arange(n, dtype=np.int64), half)
    j = rng.integers(0, n - 1, size=i.size)
    j = j + (j >= i)                                    # j != i
    a, b = np.minimum(i, j), np.maximum(i, j)
    key = np.unique(a * n + b)
    a, b = key // n, key % n
    d2 = np.sum((x[a] - x[b]) ** 2, axis=1) * (1.0 + noise * rng.standard_normal(a.size))
    d2 = np.maximum(d2, 0.0)
    r = np.concatenate([a, b])
    c = np.concatenate([b, a])
    v = np.concatenate([d2, d2])
    order = np.lexsort((c, r))
    r, c, v = r[order], c[order], v[order]
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(r, minlength=n), out=row_ptr[1:])
    return Problem("rke_n%d_pairs%d" % (n, a.size), n, n, row_ptr, c.astype(np.int32), v, lam, k0,
                   meta=dict(seed=seed, dim=dim, noise=noise, deg=deg, pattern="rke"))


@dataclass
class Request:
    arrival: float   # seconds after stream start
    m: int
    n: int
    density: float
    rank: int
    lam: float
    seed: int
    L: float = 0.0        # spectral level of the sampling and noise part of P_Omega(A)
    dsig_1: float = 0.0   # d sigma_1 and d sigma_r of the truth U V^T (d = |Omega| / (m n))
    dsig_r: float = 0.0


def truth_levels(m: int, n: int, density: float, rank: int, seed: int, noise_var: float = 0.05):
    """(L, d sigma_1, d sigma_r) of a serving request: L = sqrt(d (1 + noise var))
    (sqrt(m) + sqrt(n)), the spectral norm of P_Omega(A) - d A for unit-variance
    entries sampled with density d plus the noise, and the extreme singular
    values of the truth U V^T (drawn exactly as request_problem draws them)
    scaled by d, the size they have in P_Omega(A)."""
    nnz = max(1, int(round(density * m * n)))
    d = nnz / (m * n)
    _, U, V = values(m, n, np.zeros(m + 1, np.int64), np.zeros(1, np.int32), rank,
                     1.0 / math.sqrt(rank), noise_var, seed=seed + 7, keep_truth=True)
    sig = np.sqrt(np.maximum(np.linalg.eigvalsh((U.T @ U) @ (V.T @ V)), 0.0))
    L = math.sqrt(d * (1.0 + noise_var)) * (math.sqrt(m) + math.sqrt(n))
    return L, d * float(sig.max()), d * float(sig.min())


def serving_stream(count: int = 256, rate: float = 20.0, seed: int = 1005,
                   m_range=(500, 20_000), n_range=(1_000, 50_000), dens_range=(0.005, 0.02),
                   rank_range=(3, 15), lam_range=(0.1, 5.0), lam_over_noise=(1.0, 2.0),
                   noise_var=0.05, lam_rule: str = "levels") -> list:
    """Request descriptors of the serving workload (problems are built lazily by
    :func:`request_problem`).

    lambda, by lam_rule:
    * "levels" (the default): the midpoint of L and d sigma_r (truth_levels),
      the level of the sampling noise in P_Omega(A) and that of the weakest
      truth direction: where d sigma_r > L the solution has the truth's rank;
    * "noise": lambda = u * L with u ~ U[lam_over_noise] (above the noise only:
      a quarter of the requests then sit above d sigma_1 and end at rank 0);
    * "uniform": lambda ~ U[lam_range], which for nearly every request lies
      below L, so the solution fits the noise at ranks in the hundreds."""
    u = uniforms(seed, 0x77, 6 * count).reshape(count, 6)
    t = 0.0
    out = []
    for i in range(count):
        t += -math.log(u[i, 0]) / rate
        m = int(m_range[0] + u[i, 1] * (m_range[1] - m_range[0]))
        n = int(n_range[0] + u[i, 2] * (n_range[1] - n_range[0]))
        d = dens_range[0] + u[i, 3] * (dens_range[1] - dens_range[0])
        r = int(rank_range[0] + min(rank_range[1] - rank_range[0], int(u[i, 4] * (rank_range[1] - rank_range[0] + 1))))
        rs = seed * 1000 + i
        L, ds1, dsr = truth_levels(m, n, d, r, rs, noise_var)
        if lam_rule == "uniform":
            lam = lam_range[0] + u[i, 5] * (lam_range[1] - lam_range[0])
        elif lam_rule == "noise":
            lam = (lam_over_noise[0] + u[i, 5] * (lam_over_noise[1] - lam_over_noise[0])) * L
        elif lam_rule == "levels":
            lam = 0.5 * (L + dsr)
        else:
            raise ValueError("unknown lam_rule %r" % lam_rule)
        out.append(Request(t, m, n, d, r, lam, rs, L, ds1, dsr))
    return out


def request_problem(req: Request, k0: int = 8) -> Problem:
    nnz = max(1, int(round(req.density * req.m * req.n)))
    row_ptr, col = uniform_pattern(req.m, req.n, nnz, req.seed)
    val, _, _ = values(req.m, req.n, row_ptr, col, req.rank, 1.0 / math.sqrt(req.rank), 0.05,
                       seed=req.seed + 7)
    return Problem("req%d_%dx%d" % (req.seed, req.m, req.n), req.m, req.n, row_ptr, col, val, req.lam,
                   k0, meta=dict(seed=req.seed, rank=req.rank, pattern="uniform"))
