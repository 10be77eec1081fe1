"""GPU parity of the SPD refinement loop (the iteration of Alg. 3) through the
C-ABI, starting from a factor imported with msqrt_factor_wrap.  The factor is
the oracle's own single-precision spectral decomposition, so the comparison
isolates the HIP residual / transform / update kernels."""

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


@pytest.fixture(scope="module")
def msq():
    import paper_2607_12430_amd as m
    return m


def _truth(q, lam):
    return (q * np.sqrt(lam)[None, :]) @ q.T


@pytest.mark.parametrize("n", [1, 2, 31, 130, 257, 513])
def test_refine_from_fp32_oracle_factor(msq, n):
    torch = _torch()
    a, q, lam = W.spd(n, 1e4, 100 + n)
    lam32, q32 = oracle.syev(a.astype(np.float32), single=True)
    assert np.all(lam32 > 0)
    f = msq.factor_wrap(q32, np.sqrt(lam32).astype(np.float32), prec="fp32")
    ad = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    xd = torch.zeros_like(ad)
    info = msq.refine(f, ad, xd, init_from_factor=True, tol=1e-13)
    x = xd.cpu().numpy()
    xt = _truth(q, lam)
    # independent float64 checks on the host
    assert oracle.relres(x, a) <= 1e-13
    assert oracle.relerr(x, xt) <= 1e-11
    assert info["relres"] <= 1e-13
    assert 0 <= info["steps"] <= 3
    assert np.array_equal(x, x.T)  # symmetric-output kernels mirror exactly
    # the oracle's emulation of the same algorithm lands on the same root
    emu = oracle.emulate_mixed(a, tol=1e-13)
    assert oracle.relerr(x, emu["X"]) <= 1e-11


def test_refine_fp64_factor_needs_at_most_one_step(msq):
    torch = _torch()
    n = 200
    a, q, lam = W.spd(n, 1e4, 7)
    lam64, q64 = oracle.syev(a)
    f = msq.factor_wrap(q64, np.sqrt(lam64), prec="fp64")
    ad = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    xd = torch.zeros_like(ad)
    info = msq.refine(f, ad, xd, init_from_factor=True, tol=1e-13)
    x = xd.cpu().numpy()
    assert info["steps"] <= 1
    assert oracle.relres(x, a) <= 1e-13
    assert oracle.relerr(x, _truth(q, lam)) <= 1e-11


def test_refine_is_deterministic(msq):
    torch = _torch()
    n = 300
    a, q, lam = W.spd(n, 1e4, 8)
    lam32, q32 = oracle.syev(a.astype(np.float32), single=True)
    f = msq.factor_wrap(q32, np.sqrt(lam32).astype(np.float32), prec="fp32")
    ad = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    x1 = torch.zeros_like(ad)
    x2 = torch.zeros_like(ad)
    msq.refine(f, ad, x1)
    msq.refine(f, ad, x2)
    assert torch.equal(x1, x2)


def test_refine_from_caller_iterate_of_nearby_matrix(msq):
    # Frozen factor of A, refinement of the root of A' = A + small symmetric
    # perturbation (convergence theorem with Z != X_0).
    torch = _torch()
    n = 160
    a, q, lam = W.spd(n, 1e2, 9)
    e = W.gaussian((n, n), 10)
    e = 1e-6 * (e + e.T) / np.linalg.norm(e + e.T)
    a2 = a + e
    lam32, q32 = oracle.syev(a.astype(np.float32), single=True)
    f = msq.factor_wrap(q32, np.sqrt(lam32).astype(np.float32), prec="fp32")
    ad = torch.from_numpy(np.ascontiguousarray(a2)).cuda()
    xd = torch.from_numpy(np.ascontiguousarray(_truth(q, lam))).cuda()
    info = msq.refine(f, ad, xd, init_from_factor=False, tol=1e-13)
    x = xd.cpu().numpy()
    assert oracle.relres(x, a2) <= 1e-13
    assert oracle.relerr(x, oracle.sqrtm_spd(a2)) <= 1e-11
    assert info["steps"] >= 1


def test_refine_maxit_zero_reports_not_converged(msq):
    torch = _torch()
    n = 64
    a, q, lam = W.spd(n, 1e4, 11)
    lam32, q32 = oracle.syev(a.astype(np.float32), single=True)
    f = msq.factor_wrap(q32, np.sqrt(lam32).astype(np.float32), prec="fp32")
    ad = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    xd = torch.zeros_like(ad)
    info = msq.refine(f, ad, xd, maxit=0, allow_fail=True)
    assert info["status"] == "not_converged"
    assert info["steps"] == 0
    # X holds X_0 = Q S Q^T (float32 factor): relres around float32 level
    assert 1e-9 < info["relres"] < 1e-4
