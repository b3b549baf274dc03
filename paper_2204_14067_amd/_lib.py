"""ctypes binding of libbmg.so (include/bmg.h): argument marshalling only.

Every function here forwards to the C ABI of the same name; the arithmetic all
happens in the HIP kernels and the library's host driver.  There is no CPU
fallback: if the library is missing or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "libbmg.so")

BMG_OK, BMG_NOT_CONVERGED = 0, 1
BMG_EINVAL, BMG_ENOMEM, BMG_EDEVICE, BMG_ENONFINITE, BMG_ECANCELLED = -1, -2, -3, -4, -5
BMG_FP64, BMG_FP32, BMG_BF16 = 0, 1, 2
BMG_STEP_FIXED, BMG_STEP_SPARSA = 0, 1
BMG_BM_PSD, BMG_BM_POLYMF = 0, 1
STATUS_NAMES = {0: "BMG_OK", 1: "BMG_NOT_CONVERGED", -1: "BMG_EINVAL", -2: "BMG_ENOMEM",
                -3: "BMG_EDEVICE", -4: "BMG_ENONFINITE", -5: "BMG_ECANCELLED"}

# the C ABI's exported entry points (checked by the CPU tests)
EXPORTS = ["bmg_options_default", "bmg_workspace_size", "bmg_problem_create", "bmg_problem_destroy",
           "bmg_sddmm", "bmg_spmm", "bmg_bm_epochs", "bmg_polymf_epochs", "bmg_objective",
           "bmg_prox_step", "bmg_solve", "bmg_rke_residual", "bmg_rke_solve",
           "bmg_last_error", "bmg_server_footprint", "bmg_server_create", "bmg_server_submit",
           "bmg_server_poll", "bmg_server_drain", "bmg_server_stats", "bmg_server_batch_stats",
           "bmg_server_destroy", "bmg_server_tick", "bmg_sddmm_static"]


class BmgCsr(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class BmgOptions(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("alpha", ctypes.c_double), ("tol", ctypes.c_double),
                ("ssi_tol_floor", ctypes.c_double), ("psi0", ctypes.c_double),
                ("bm_epochs", ctypes.c_int), ("max_iter", ctypes.c_int),
                ("ssi_max_iter", ctypes.c_int), ("k_init", ctypes.c_int),
                ("refresh_every", ctypes.c_int), ("verbose", ctypes.c_int),
                ("timing", ctypes.c_int), ("lmsvd_p", ctypes.c_int),
                ("seed", ctypes.c_uint64), ("step_rule", ctypes.c_int), ("bm_solver", ctypes.c_int),
                ("alpha_min", ctypes.c_double), ("alpha_max", ctypes.c_double),
                ("sparsa_beta", ctypes.c_double), ("sparsa_delta", ctypes.c_double),
                ("dense_rows", ctypes.c_double)]


class BmgResult(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int), ("iters", ctypes.c_int), ("ssi_iters", ctypes.c_int),
                ("status", ctypes.c_int), ("F", ctypes.c_double), ("F_bm", ctypes.c_double),
                ("residual", ctypes.c_double), ("eps", ctypes.c_double),
                ("seconds", ctypes.c_double), ("sparse_bytes", ctypes.c_double),
                ("sparse_passes", ctypes.c_int), ("kernel_ms", ctypes.c_double * 3),
                ("kernel_bytes", ctypes.c_double * 3), ("kernel_launches", ctypes.c_int * 3),
                ("host_la_seconds", ctypes.c_double), ("host_wait_seconds", ctypes.c_double),
                ("host_syncs", ctypes.c_int), ("pg_trials", ctypes.c_int),
                ("alpha_last", ctypes.c_double), ("bf16_passes", ctypes.c_int)]

    def as_dict(self):
        out = {}
        for f, _ in self._fields_:
            v = getattr(self, f)
            out[f] = list(v) if hasattr(v, "_length_") else v
        return out


class BmgRequestInfo(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int), ("status", ctypes.c_int), ("k", ctypes.c_int),
                ("queued_s", ctypes.c_double), ("run_s", ctypes.c_double),
                ("total_s", ctypes.c_double), ("footprint", ctypes.c_size_t),
                ("result", BmgResult)]


class BmgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


_lib = None


def load():
    """Load libbmg.so (it must have been built: python -m paper_2204_14067_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(SO):
        raise ImportError("libbmg.so is not built (%s); run python -m paper_2204_14067_amd.build" % SO)
    lib = ctypes.CDLL(SO)
    p, i32, i64, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    lib.bmg_options_default.argtypes = [P(BmgOptions)]
    lib.bmg_options_default.restype = None
    lib.bmg_workspace_size.argtypes = [i64, i64, i64, i32, i32, P(BmgOptions), P(ctypes.c_size_t)]
    lib.bmg_problem_create.argtypes = [P(BmgCsr), i32, i32, P(BmgOptions), p, ctypes.c_size_t, p, P(p)]
    lib.bmg_problem_destroy.argtypes = [p]
    lib.bmg_problem_destroy.restype = None
    lib.bmg_sddmm.argtypes = [p, p, p, i32, i32, p, P(d)]
    lib.bmg_spmm.argtypes = [p, p, p, i32, i32, p, i32, i32]
    lib.bmg_bm_epochs.argtypes = [p, p, p, i32, i32, d, i32, P(d)]
    lib.bmg_polymf_epochs.argtypes = [p, p, p, i32, i32, d, i32, P(d)]
    lib.bmg_rke_residual.argtypes = [p, p, i32, i32, p, p, P(d)]
    lib.bmg_rke_solve.argtypes = [p, p, i32, P(BmgOptions), P(i32), P(BmgResult)]
    lib.bmg_objective.argtypes = [p, p, p, i32, i32, d, P(d), P(d)]
    lib.bmg_prox_step.argtypes = [p, p, p, P(i32), i32, P(BmgOptions), P(d), P(d)]
    lib.bmg_solve.argtypes = [p, p, p, i32, P(BmgOptions), P(i32), P(BmgResult)]
    lib.bmg_server_footprint.argtypes = [i64, i64, i64, i32, i32, P(BmgOptions), P(ctypes.c_size_t)]
    lib.bmg_server_create.argtypes = [p, ctypes.c_size_t, i32, i32, P(p)]
    lib.bmg_server_tick.argtypes = [p, P(i32), P(i32)]
    lib.bmg_server_submit.argtypes = [p, P(BmgCsr), i32, i32, P(BmgOptions), P(ctypes.c_uint64)]
    lib.bmg_server_poll.argtypes = [p, ctypes.c_uint64, P(BmgRequestInfo), p, p, i32]
    lib.bmg_server_drain.argtypes = [p]
    lib.bmg_server_stats.argtypes = [p, P(i32), P(ctypes.c_size_t)]
    lib.bmg_server_batch_stats.argtypes = [p, P(i64), P(i64)]
    lib.bmg_server_destroy.argtypes = [p]
    lib.bmg_server_destroy.restype = None
    lib.bmg_sddmm_static.argtypes = [P(BmgCsr), p, p, i32, i32, p, P(d), p]
    for f in ["bmg_workspace_size", "bmg_problem_create", "bmg_sddmm", "bmg_spmm", "bmg_bm_epochs",
              "bmg_polymf_epochs", "bmg_rke_residual", "bmg_rke_solve",
              "bmg_objective", "bmg_prox_step", "bmg_solve", "bmg_server_footprint",
              "bmg_server_create", "bmg_server_submit", "bmg_server_poll", "bmg_server_drain",
              "bmg_server_stats", "bmg_server_batch_stats", "bmg_sddmm_static", "bmg_server_tick"]:
        getattr(lib, f).restype = ctypes.c_int
    lib.bmg_last_error.argtypes = []
    lib.bmg_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def check(status, allow=(BMG_OK,)):
    if status not in allow:
        raise BmgError(status, load().bmg_last_error().decode())
    return status
