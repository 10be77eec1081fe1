"""BF16-split precision class: the split MFMA product against a float64
reference (unit roundoff about 2^-16 of |A||B|, visibly coarser than the
float product), and complete solves with prec="bf16split" meeting the same
residual and forward-error bounds as the other precisions."""

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


def _msq():
    import paper_2607_12430_amd as msq
    return msq


@pytest.mark.parametrize("ta,tb", [(False, False), (True, False), (False, True), (True, True)])
@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (33, 17, 5), (128, 128, 32), (257, 130, 300),
                                   (500, 64, 1000)])
def test_split_gemm_accuracy(ta, tb, m, n, k):
    msq = _msq()
    rng = np.random.Generator(np.random.PCG64(m * 7 + n * 3 + k))
    a = rng.standard_normal((k, m) if ta else (m, k)).astype(np.float32)
    b = rng.standard_normal((n, k) if tb else (k, n)).astype(np.float32)
    a64 = a.astype(np.float64).T if ta else a.astype(np.float64)
    b64 = b.astype(np.float64).T if tb else b.astype(np.float64)
    ref = a64 @ b64
    scale = np.abs(a64) @ np.abs(b64)
    c_split = msq.test_gemm_f32(a, b, split=True, ta=ta, tb=tb).astype(np.float64)
    c_f32 = msq.test_gemm_f32(a, b, split=False, ta=ta, tb=tb).astype(np.float64)
    err_split = np.max(np.abs(c_split - ref) / scale)
    err_f32 = np.max(np.abs(c_f32 - ref) / scale)
    # hi*hi + hi*lo + lo*hi drops lo*lo and the split remainder: ~2^-16
    assert err_split <= 3.0 * 2.0 ** -16
    assert err_f32 <= 4.0 * k * 2.0 ** -24 + 1e-30
    if k >= 32:
        # the split product is the coarser one: the flag really selects it
        assert err_split > err_f32


@pytest.mark.parametrize("n,kappa", [(64, 1e2), (300, 1e2), (513, 1e3)])
def test_spd_bf16split_solve(n, kappa):
    import torch
    msq = _msq()
    a, q, lam = W.spd(n, kappa, 501 + n)
    x_true = (q * np.sqrt(lam)) @ q.T
    at = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    x, info = msq.sqrtm(at, prec="bf16split", fallback=False)
    _, i32 = msq.sqrtm(at, prec="fp32", fallback=False)
    x = x.cpu().numpy()
    assert info["prec_used"] == "bf16split"
    assert info["relres"] <= 1e-13
    assert oracle.relres(x, a) <= 1e-13
    assert oracle.relerr(x, x_true) <= 1e-11
    # coarser transforms need at least as many corrections as float ones
    assert info["steps"] >= i32["steps"]


@pytest.mark.parametrize("n", [40, 150])
def test_general_bf16split_solve(n):
    import torch
    msq = _msq()
    a = W.nonsym_shifted(n, 601 + n)
    x, info = msq.sqrtm(torch.from_numpy(np.ascontiguousarray(a)).cuda(), prec="bf16split",
                        fallback=False)
    x = x.cpu().numpy()
    assert info["prec_used"] == "bf16split"
    assert info["relres"] <= 1e-13
    assert oracle.relerr(x, oracle.sqrtm(a)) <= 1e-11
