"""BM-Global nuclear-norm matrix completion on one MI355X (gfx950).

Thin Python front end of libbmg.so (C ABI in include/bmg.h).  PyTorch supplies
device memory and the HIP stream; every step of the method runs in the
library's HIP kernels and host driver.

    import torch, paper_2204_14067_amd as bmg
    prob = bmg.Problem(row_ptr, col, val, m, n, k_cap=64)      # device tensors
    W, H, k, res = prob.bmg_solve(lam=0.5, k_init=8, tol=1e-6)

Method names mirror the C entry points (bmg_sddmm, bmg_spmm, bmg_bm_epochs,
bmg_objective, bmg_prox_step, bmg_solve).
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import (BMG_BF16, BMG_FP32, BMG_FP64, BMG_NOT_CONVERGED, BMG_OK, BmgError,  # noqa: F401
                   BmgOptions, BmgResult)

_PREC = {"fp64": BMG_FP64, "fp32": BMG_FP32, "bf16": BMG_BF16}


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream_handle(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def options(**kw) -> BmgOptions:
    """bmg_options with the library defaults, overridden by keyword (lam= sets
    lambda; step_rule= takes "fixed" / "sparsa" or the enum value)."""
    o = BmgOptions()
    _lib.load().bmg_options_default(ctypes.byref(o))
    for key, v in kw.items():
        if key == "step_rule" and isinstance(v, str):
            v = {"fixed": _lib.BMG_STEP_FIXED, "sparsa": _lib.BMG_STEP_SPARSA}[v]
        if key == "bm_solver" and isinstance(v, str):
            v = {"psd": _lib.BMG_BM_PSD, "polymf": _lib.BMG_BM_POLYMF}[v]
        if not hasattr(o, "lambda_" if key in ("lam", "lambda") else key):
            raise TypeError("unknown option %r" % key)
        setattr(o, "lambda_" if key in ("lam", "lambda") else key, v)
    return o


def round_ld(k: int) -> int:
    return max(8, (k + 7) // 8 * 8)


class Problem:
    """One completion problem resident on the GPU (bmg_problem_create).

    row_ptr (int64, m+1), col (int32, nnz), val (float64, nnz) are device
    tensors that must stay alive; the workspace is a torch allocation owned by
    this object.  lmsvd_p / sparsa reserve workspace for solves with that many
    LmSVD history blocks / with the SpaRSA step rule (bmg_workspace_size);
    dense_rows > 0 moves the rows at least that dense into a dense panel."""

    def __init__(self, row_ptr, col, val, m: int, n: int, k_cap: int = 64, precision: str = "fp64",
                 device=None, lmsvd_p: int = 0, sparsa: bool = False, dense_rows: float = 0.0):
        lib = _lib.load()
        if not torch.cuda.is_available():
            raise RuntimeError("paper_2204_14067_amd needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.device = torch.device(device) if device is not None else row_ptr.device
        assert row_ptr.is_cuda and col.is_cuda and val.is_cuda
        assert row_ptr.dtype == torch.int64 and col.dtype == torch.int32 and val.dtype == torch.float64
        self.row_ptr, self.col, self.val = row_ptr.contiguous(), col.contiguous(), val.contiguous()
        self.m, self.n, self.nnz, self.k_cap = int(m), int(n), int(col.numel()), int(k_cap)
        self.precision = _PREC[precision]
        nbytes = ctypes.c_size_t(0)
        self.reserve = options(lmsvd_p=lmsvd_p, step_rule="sparsa" if sparsa else "fixed",
                               dense_rows=dense_rows)
        _lib.check(lib.bmg_workspace_size(self.m, self.n, self.nnz, self.k_cap, self.precision,
                                          ctypes.byref(self.reserve), ctypes.byref(nbytes)))
        self.ws = torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8, device=self.device)
        csr = _lib.BmgCsr(self.m, self.n, self.nnz, self.row_ptr.data_ptr(), self.col.data_ptr(),
                          self.val.data_ptr())
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(lib.bmg_problem_create(ctypes.byref(csr), self.k_cap, self.precision,
                                              ctypes.byref(self.reserve), _ptr(self.ws), self.ws.numel(),
                                              _stream_handle(self.device), ctypes.byref(h)))
        self._h = h
        self.ld = round_ld(self.k_cap)

    @classmethod
    def from_host(cls, row_ptr, col, val, m, n, k_cap=64, precision="fp64", device="cuda:0",
                  lmsvd_p=0, sparsa=False, dense_rows=0.0):
        t = lambda a, dt: torch.as_tensor(a).to(device=device, dtype=dt).contiguous()  # noqa: E731
        return cls(t(row_ptr, torch.int64), t(col, torch.int32), t(val, torch.float64), m, n, k_cap,
                   precision, device, lmsvd_p=lmsvd_p, sparsa=sparsa, dense_rows=dense_rows)

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().bmg_problem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _factors(self, W, H, k):
        ld = W.shape[1]
        assert W.dtype == torch.float64 and H.dtype == torch.float64 and W.is_cuda and H.is_cuda
        assert W.shape == (self.m, ld) and H.shape == (self.n, ld) and W.is_contiguous() and H.is_contiguous()
        return ld

    def zeros_factors(self, ld=None):
        ld = ld or self.ld
        return (torch.zeros(self.m, ld, dtype=torch.float64, device=self.device),
                torch.zeros(self.n, ld, dtype=torch.float64, device=self.device))

    # ------------------------------------------------------------------ entry points
    def bmg_sddmm(self, W, H, k, R=None, store=True):
        ld = self._factors(W, H, k)
        if R is None and store:
            R = torch.empty(self.nnz, dtype=torch.float64, device=self.device)
        hs = ctypes.c_double(0.0)
        _lib.check(_lib.load().bmg_sddmm(self._h, _ptr(W), _ptr(H), k, ld, _ptr(R), ctypes.byref(hs)))
        return R, hs.value

    def bmg_spmm(self, S, B, transpose=False, C=None):
        q = B.shape[1]
        rows = self.n if transpose else self.m
        if C is None:
            C = torch.empty(rows, B.shape[1], dtype=torch.float64, device=self.device)
        _lib.check(_lib.load().bmg_spmm(self._h, _ptr(S), _ptr(B), q, B.stride(0), _ptr(C), C.stride(0),
                                        1 if transpose else 0))
        return C

    def bmg_bm_epochs(self, W, H, k, lam, epochs=1):
        ld = self._factors(W, H, k)
        F = ctypes.c_double(0.0)
        _lib.check(_lib.load().bmg_bm_epochs(self._h, _ptr(W), _ptr(H), k, ld, lam, epochs,
                                             ctypes.byref(F)))
        return F.value

    def bmg_polymf_epochs(self, W, H, k, lam, epochs=1):
        ld = self._factors(W, H, k)
        F = ctypes.c_double(0.0)
        _lib.check(_lib.load().bmg_polymf_epochs(self._h, _ptr(W), _ptr(H), k, ld, lam, epochs,
                                                 ctypes.byref(F)))
        return F.value

    def bmg_objective(self, W, H, k, lam, residual=False):
        """F at X = W H^T; with residual=True also the relative optimality
        residual there (one inexact PG step, the factors untouched): (F, res)."""
        ld = self._factors(W, H, k)
        F = ctypes.c_double(0.0)
        res = ctypes.c_double(0.0)
        _lib.check(_lib.load().bmg_objective(self._h, _ptr(W), _ptr(H), k, ld, lam, ctypes.byref(F),
                                             ctypes.byref(res) if residual else None))
        return (F.value, res.value) if residual else F.value

    def bmg_prox_step(self, W, H, k, **opts):
        ld = self._factors(W, H, k)
        o = options(**opts)
        kk = ctypes.c_int(k)
        sig = (ctypes.c_double * max(self.k_cap, 1))()
        res = ctypes.c_double(0.0)
        _lib.check(_lib.load().bmg_prox_step(self._h, _ptr(W), _ptr(H), ctypes.byref(kk), ld,
                                             ctypes.byref(o), sig, ctypes.byref(res)))
        return kk.value, [sig[i] for i in range(kk.value)], res.value

    def bmg_solve(self, W=None, H=None, **opts):
        o = options(**opts)
        if W is None:
            W, H = self.zeros_factors()
        ld = self._factors(W, H, 0)
        k = ctypes.c_int(0)
        r = BmgResult()
        st = _lib.load().bmg_solve(self._h, _ptr(W), _ptr(H), ld, ctypes.byref(o), ctypes.byref(k),
                                   ctypes.byref(r))
        _lib.check(st, allow=(BMG_OK, BMG_NOT_CONVERGED))
        return W, H, k.value, r.as_dict()

    # -------------------------------------------------------------- kernel-estimation QSDP
    def bmg_rke_residual(self, W, k):
        """(r in CSR order, row sums of r, sum r^2) at X = W W^T (symmetric Omega)."""
        ld = W.stride(0)
        r = torch.empty(max(self.nnz, 1), dtype=torch.float64, device=self.device)
        deg = torch.empty(max(self.n, 1), dtype=torch.float64, device=self.device)
        s2 = ctypes.c_double(0.0)
        _lib.check(_lib.load().bmg_rke_residual(self._h, _ptr(W), k, ld, _ptr(r), _ptr(deg),
                                                ctypes.byref(s2)))
        return r[:self.nnz], deg[:self.n], s2.value

    def bmg_rke_solve(self, **opts):
        """BM-Global on the kernel-estimation QSDP; returns (W, k, result dict)."""
        o = options(**opts)
        W = torch.zeros((self.n, round_ld(self.k_cap)), dtype=torch.float64, device=self.device)
        k = ctypes.c_int(0)
        r = BmgResult()
        st = _lib.load().bmg_rke_solve(self._h, _ptr(W), W.stride(0), ctypes.byref(o), ctypes.byref(k),
                                       ctypes.byref(r))
        _lib.check(st, allow=(BMG_OK, BMG_NOT_CONVERGED))
        return W, k.value, r.as_dict()


def bmg_sddmm_static(row_ptr, col, val, m, n, W, H, k, R=None, store=True):
    """bmg_sddmm without a problem object or workspace (the library's static
    device scratch; for callers that cannot allocate).  Device tensors: row_ptr
    int64 [m+1], col int32 [nnz], val float64 [nnz], W (m x ld), H (n x ld)
    float64.  Returns (R or None, 1/2 sum R^2)."""
    lib = _lib.load()
    ld = W.shape[1]
    assert W.dtype == torch.float64 and H.dtype == torch.float64 and H.shape[1] == ld
    assert W.is_contiguous() and H.is_contiguous()
    nnz = int(col.numel())
    if R is None and store:
        R = torch.empty(max(nnz, 1), dtype=torch.float64, device=W.device)
    csr = _lib.BmgCsr(int(m), int(n), nnz, row_ptr.data_ptr(), col.data_ptr(), val.data_ptr())
    hs = ctypes.c_double(0.0)
    with torch.cuda.device(W.device):
        _lib.check(lib.bmg_sddmm_static(ctypes.byref(csr), _ptr(W), _ptr(H), k, ld, _ptr(R),
                                        ctypes.byref(hs), _stream_handle(W.device)))
    return (R[:nnz] if R is not None else None), hs.value


class Server:
    """Request loop over many problems on one GPU (bmg_server_*): admission by
    HBM footprint inside one torch-allocated arena, max_slots problems running
    concurrently on their own streams.  threads=True: worker threads solve the
    admitted problems; threads=False: the caller drives it with tick()."""

    def __init__(self, arena_bytes: int, max_slots: int = 4, device="cuda:0", threads: bool = True):
        lib = _lib.load()
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        with torch.cuda.device(torch.device(device)):
            _lib.check(lib.bmg_server_create(_ptr(self.arena), self.arena.numel(), max_slots,
                                             1 if threads else 0, ctypes.byref(h)))
        self._h = h

    @staticmethod
    def footprint(m, n, nnz, k_cap=64, precision="fp32", **opts):
        """Arena bytes of one request (opts as for submit: lmsvd_p and step_rule
        size its workspace)."""
        b = ctypes.c_size_t(0)
        o = options(**opts)
        _lib.check(_lib.load().bmg_server_footprint(m, n, nnz, k_cap, _PREC[precision], ctypes.byref(o),
                                                    ctypes.byref(b)))
        return b.value

    def submit(self, row_ptr, col, val, m, n, k_cap=64, precision="fp32", **opts):
        import numpy as np
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        cl = np.ascontiguousarray(col, dtype=np.int32)
        vl = np.ascontiguousarray(val, dtype=np.float64)
        csr = _lib.BmgCsr(m, n, len(cl), rp.ctypes.data, cl.ctypes.data, vl.ctypes.data)
        o = options(**opts)
        t = ctypes.c_uint64(0)
        _lib.check(_lib.load().bmg_server_submit(self._h, ctypes.byref(csr), k_cap, _PREC[precision],
                                                 ctypes.byref(o), ctypes.byref(t)))
        return t.value

    def poll(self, ticket, m=None, n=None, ld=None):
        import numpy as np
        info = _lib.BmgRequestInfo()
        W = H = None
        wp = hp = None
        if m is not None:
            W = np.zeros((m, ld)); H = np.zeros((n, ld))
            wp, hp = W.ctypes.data_as(ctypes.c_void_p), H.ctypes.data_as(ctypes.c_void_p)
        _lib.check(_lib.load().bmg_server_poll(self._h, ticket, ctypes.byref(info), wp, hp, ld or 0))
        out = {"state": info.state, "status": info.status, "k": info.k, "queued_s": info.queued_s,
               "run_s": info.run_s, "total_s": info.total_s, "footprint": info.footprint,
               "result": info.result.as_dict()}
        return out, W, H

    def tick(self):
        """bmg_server_tick: (running, queued) after one round."""
        r, q = ctypes.c_int(0), ctypes.c_int(0)
        _lib.check(_lib.load().bmg_server_tick(self._h, ctypes.byref(r), ctypes.byref(q)))
        return r.value, q.value

    def drain(self):
        _lib.check(_lib.load().bmg_server_drain(self._h))

    def stats(self):
        pr, pb = ctypes.c_int(0), ctypes.c_size_t(0)
        _lib.check(_lib.load().bmg_server_stats(self._h, ctypes.byref(pr), ctypes.byref(pb)))
        bl, bp = ctypes.c_int64(0), ctypes.c_int64(0)
        _lib.check(_lib.load().bmg_server_batch_stats(self._h, ctypes.byref(bl), ctypes.byref(bp)))
        return {"peak_running": pr.value, "peak_bytes": pb.value, "shared_launches": bl.value,
                "batched_passes": bp.value}

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().bmg_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
