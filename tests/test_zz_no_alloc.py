"""The allocation-free entry point bmg_sddmm_static (static device scratch, no
problem object, no workspace) against bmg_sddmm on a problem built from the
same CSR, and against the oracle: two calls in a row, the second on a smaller
input, so the second call runs on scratch the first one left behind.

R is compared bit for bit with bmg_sddmm (both take each entry's dot product
in the same lane layout); half_sq adds the same terms in another order, so it
is held to relative 1e-12 against bmg_sddmm and against the oracle's sum."""
import math

import numpy as np
import pytest
import torch

import paper_2204_14067_amd as bmg
import synth
from oracle import core

pytestmark = pytest.mark.gpu
U = 2.0 ** -53
DEV = "cuda:0"


def _dev(a, dt):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=DEV, dtype=dt).contiguous()


def _run(p, k, seed):
    print("sddmm_static", p.name, p.m, p.n, p.nnz, "k", k, flush=True)
    ld = bmg.round_ld(k)
    rng = np.random.default_rng(seed)
    W = np.zeros((p.m, ld)); H = np.zeros((p.n, ld))
    W[:, :k] = rng.standard_normal((p.m, k))
    H[:, :k] = rng.standard_normal((p.n, k))
    rp, cl, vl = _dev(p.row_ptr, torch.int64), _dev(p.col, torch.int32), _dev(p.val, torch.float64)
    Wd, Hd = _dev(W, torch.float64), _dev(H, torch.float64)
    R_s, hs_s = bmg.bmg_sddmm_static(rp, cl, vl, p.m, p.n, Wd, Hd, k)
    torch.cuda.synchronize()
    dp = bmg.Problem(rp, cl, vl, p.m, p.n, k_cap=max(k, 8))
    R_p, hs_p = dp.bmg_sddmm(Wd, Hd, k)
    torch.cuda.synchronize()
    R_s, R_p = R_s.cpu().numpy(), R_p.cpu().numpy()
    assert np.array_equal(R_s, R_p)
    assert math.isclose(hs_s, hs_p, rel_tol=1e-12, abs_tol=1e-300)
    Ro = core.sddmm(p, W[:, :k], H[:, :k])
    bound = 4 * k * U * (core.sddmm(p, np.abs(W[:, :k]), np.abs(H[:, :k]), with_values=False)
                         + np.abs(p.val))
    assert np.all(np.abs(R_s - Ro) <= bound + 1e-300)
    assert math.isclose(hs_s, 0.5 * float(np.sum(Ro ** 2)), rel_tol=1e-12, abs_tol=1e-300)
    dp.close()
    return hs_s


def test_static_matches_bmg_sddmm_twice_second_smaller():
    big = synth.netflix_shape(scale=0.03)          # power law: rows far longer than 2048 entries
    small = synth.tiny(90, 35, 900, seed=5)         # m > n, far fewer rows
    _run(big, 33, seed=1)
    _run(small, 17, seed=2)


def test_static_edge_cases():
    _run(synth.tiny(80, 50, 40, seed=4), 5, seed=3)     # empty rows
    _run(synth.tiny(3, 4, 1), 1, seed=4)                # one entry
    _run(synth.tiny(7, 11, 30), 200, seed=5)            # 16-lane groups


def test_static_rejects_bad_csr_and_oversize():
    p = synth.tiny(7, 11, 30)
    bad = p.col.copy()
    bad[3] = 11                                          # column out of range
    W = torch.zeros(p.m, 8, dtype=torch.float64, device=DEV)
    H = torch.zeros(p.n, 8, dtype=torch.float64, device=DEV)
    args = (_dev(p.row_ptr, torch.int64), _dev(bad, torch.int32), _dev(p.val, torch.float64))
    with pytest.raises(bmg.BmgError, match="out of range"):
        bmg.bmg_sddmm_static(*args, p.m, p.n, W, H, 4)
    # the call after a rejected one starts from a cleared flag
    good = (_dev(p.row_ptr, torch.int64), _dev(p.col, torch.int32), _dev(p.val, torch.float64))
    _, hs = bmg.bmg_sddmm_static(*good, p.m, p.n, W, H, 4)
    assert math.isclose(hs, 0.5 * float(np.sum(p.val ** 2)), rel_tol=1e-12)
