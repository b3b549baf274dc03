"""Host-side checks that need no GPU: the C-ABI library loads and exports every
entry point include/bmg.h declares; host queries validate their arguments;
the synthetic generators are deterministic and produce valid CSR."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.abspath(os.path.join(os.path.dirname(__file__), ".."))


def header_functions():
    text = open(os.path.join(ROOT, "include", "bmg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bmg_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2204_14067_amd import _lib
    if not os.path.exists(_lib.SO):
        from paper_2204_14067_amd import build
        build.build()
    return _lib.load()


def test_library_exports_every_declared_symbol(lib):
    from paper_2204_14067_amd import _lib
    names = header_functions()
    assert len(names) >= 11
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(_lib.EXPORTS) == names


def test_options_default(lib):
    from paper_2204_14067_amd import _lib
    o = _lib.BmgOptions()
    o.lmsvd_p, o.seed, o.timing = 7, 123, 1
    lib.bmg_options_default(ctypes.byref(o))
    assert o.alpha == 1.99 and o.bm_epochs == 3 and o.psi0 == 0.1 and o.tol == 1e-6
    assert o.k_init == 8 and o.refresh_every == 5 and o.ssi_max_iter == 50
    assert o.lmsvd_p == 0 and o.seed == 0 and o.timing == 0
    assert o.step_rule == _lib.BMG_STEP_FIXED and o.alpha_min == 1.99 and o.alpha_max == 1e3
    assert o.sparsa_beta == 0.5 and o.sparsa_delta == 0.999


def test_workspace_size_and_argument_checks(lib):
    from paper_2204_14067_amd import _lib
    nb = ctypes.c_size_t(0)
    assert lib.bmg_workspace_size(1000, 1500, 50_000, 128, _lib.BMG_FP64, None, ctypes.byref(nb)) == 0
    small = nb.value
    assert small > 50_000 * 36
    assert lib.bmg_workspace_size(1000, 1500, 500_000, 128, _lib.BMG_FP64, None, ctypes.byref(nb)) == 0
    assert nb.value > small
    assert lib.bmg_workspace_size(-1, 5, 5, 8, 0, None, ctypes.byref(nb)) == _lib.BMG_EINVAL
    assert b"bad shape" in lib.bmg_last_error()
    assert lib.bmg_workspace_size(10, 10, 5, 0, 0, None, ctypes.byref(nb)) == _lib.BMG_EINVAL
    assert lib.bmg_workspace_size(10, 10, 5, 4096, 0, None, ctypes.byref(nb)) == _lib.BMG_EINVAL
    # creating with a null CSR is rejected before any device call
    h = ctypes.c_void_p()
    assert lib.bmg_problem_create(None, 8, 0, None, None, 0, None, ctypes.byref(h)) == _lib.BMG_EINVAL


def test_workspace_reserves_history_and_sparsa_state(lib):
    """The workspace grows by exactly the regions the solver variants need:
    (2p - 1) short-side and 3p long-side blocks of qb columns for p history
    blocks, and for SpaRSA one short-side block, (m + n) rows at ld_k and two
    nnz-vectors (FP64 here, qb = 2 k_cap + 2 and ld_k = k_cap, both rounded up to
    16, every region rounded up to 256 bytes)."""
    from paper_2204_14067_amd import _lib
    m, n, nnz, kc = 1000, 1500, 50_000, 40
    qb, ldk = (2 * kc + 2 + 15) // 16 * 16, (kc + 15) // 16 * 16
    r256 = lambda b: (b + 255) // 256 * 256                        # noqa: E731
    size = {}
    for p_, rule in ((0, 0), (1, 0), (3, 0), (0, 1)):
        o = _lib.BmgOptions()
        lib.bmg_options_default(ctypes.byref(o))
        o.lmsvd_p, o.step_rule = p_, rule
        nb = ctypes.c_size_t(0)
        assert lib.bmg_workspace_size(m, n, nnz, kc, _lib.BMG_FP64, ctypes.byref(o), ctypes.byref(nb)) == 0
        size[(p_, rule)] = nb.value
    base = size[(0, 0)]
    mb, lb = r256(8 * m * qb), r256(8 * n * qb)
    # every region is rounded up to a multiple of 256 bytes plus one guard unit
    for p_ in (1, 3):
        need = (2 * p_ - 1) * mb + 3 * p_ * lb
        assert need <= size[(p_, 0)] - base <= need + 256
    sp = r256(8 * m * qb) + r256(8 * m * ldk) + r256(8 * n * ldk) + 2 * r256(8 * nnz)
    assert sp <= size[(0, 1)] - base <= sp + 256
    o = _lib.BmgOptions()
    lib.bmg_options_default(ctypes.byref(o))
    o.lmsvd_p = 5
    nb = ctypes.c_size_t(0)
    assert lib.bmg_workspace_size(m, n, nnz, kc, _lib.BMG_FP64, ctypes.byref(o), ctypes.byref(nb)) == _lib.BMG_EINVAL


def test_no_cpu_fallback_without_gpu():
    import torch
    import paper_2204_14067_amd as bmg
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    p = synth.tiny(5, 6, 10)
    with pytest.raises(RuntimeError):
        bmg.Problem(torch.as_tensor(p.row_ptr), torch.as_tensor(p.col), torch.as_tensor(p.val),
                    p.m, p.n)


def _check_csr(p):
    assert p.row_ptr[0] == 0 and p.row_ptr[-1] == len(p.col) == len(p.val)
    assert np.all(np.diff(p.row_ptr) >= 0)
    assert p.col.min(initial=0) >= 0 and (len(p.col) == 0 or p.col.max() < p.n)
    rows = p.rows()
    key = rows * p.n + p.col
    assert np.all(np.diff(key) > 0)   # sorted, duplicate-free


def test_synth_uniform_and_powerlaw_valid_and_deterministic():
    a = synth.small_uniform()
    _check_csr(a)
    assert a.nnz == 50_000 and a.m == 1000 and a.n == 1500
    b = synth.small_uniform()
    assert np.array_equal(a.col, b.col) and np.array_equal(a.val, b.val)
    p = synth.netflix_shape(scale=0.05)
    _check_csr(p)
    deg = np.diff(p.row_ptr)
    assert deg.max() > 20 * np.median(deg)          # heavy-tailed rows
    assert p.val.min() >= 1.0 and p.val.max() <= 5.0  # ratings clip
    q = synth.netflix_shape(scale=0.05)
    assert np.array_equal(p.col, q.col)


def test_serving_stream_shapes():
    reqs = synth.serving_stream(count=64)
    t = [r.arrival for r in reqs]
    assert all(b > a for a, b in zip(t, t[1:]))
    assert 1.0 < t[-1] < 8.0          # ~64 / 20 per second
    assert all(500 <= r.m <= 20000 and 1000 <= r.n <= 50000 and 3 <= r.rank <= 15 for r in reqs)


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_static_sddmm_rejects_oversize_before_device_work(lib):
    """bmg_sddmm_static refuses more rows than its static scratch covers before
    it touches the device (so this runs without a GPU)."""
    from paper_2204_14067_amd import _lib
    csr = _lib.BmgCsr(600_000, 10, 0, None, None, None)
    hs = ctypes.c_double(-1.0)
    st = lib.bmg_sddmm_static(ctypes.byref(csr), None, None, 0, 8, None, ctypes.byref(hs), None)
    assert st == _lib.BMG_ENOMEM
    assert b"static scratch" in lib.bmg_last_error()
    csr = _lib.BmgCsr(10, 10, 0, None, None, None)
    assert lib.bmg_sddmm_static(ctypes.byref(csr), None, None, 300, 304, None, None, None) == _lib.BMG_EINVAL
