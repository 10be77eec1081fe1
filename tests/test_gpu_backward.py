"""GPU parity of the backward solve X G + G X = Gbar (msqrt_sqrtm_backward and
the autograd wrapper) against the oracle's closed-form adjoint, Kronecker
brute force and central differences of the forward solve."""

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def msq():
    import paper_2607_12430_amd as m
    return m


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("n", [1, 8, 65, 200])
def test_backward_matches_closed_form(msq, n, prec):
    a, q, lam = W.spd(n, 1e4, 600 + n)
    gbar = W.gaussian((n, n), 700 + n)
    x, info, f = msq.sqrtm(_dev(a), prec=prec, keep_factor=True, fallback=False)
    g, binfo = msq.sqrtm_backward(f, x, _dev(gbar))
    g = g.cpu().numpy()
    ref = oracle.adjoint_spd(q, lam, gbar)
    assert oracle.relerr(g, ref) <= 1e-10
    assert binfo["relres"] <= 1e-13
    if n <= 8:
        xr = (q * np.sqrt(lam)) @ q.T
        assert oracle.relerr(g, oracle.kron_adjoint(xr, gbar).real) <= 1e-10


def test_backward_central_differences(msq):
    n = 48
    a, q, lam = W.spd(n, 1e2, 11)
    gbar = W.gaussian((n, n), 12)
    x, _, f = msq.sqrtm(_dev(a), keep_factor=True)
    g = msq.sqrtm_backward(f, x, _dev(gbar))[0].cpu().numpy()
    h = 1e-6
    for seed in (300, 301, 302):
        z = W.gaussian((n, n), seed)
        e = (z + z.T) / np.linalg.norm(z + z.T)
        xp = msq.sqrtm(_dev(a + h * e))[0].cpu().numpy()
        xm = msq.sqrtm(_dev(a - h * e))[0].cpu().numpy()
        fd = np.sum(gbar * (xp - xm)) / (2 * h)
        assert abs(fd - np.sum(g * e)) <= 1e-6 * max(1.0, abs(fd))


def test_batched_forward_and_backward(msq):
    # 16 x n=128 (the 64 x 512 workload at full size is in test_configs)
    import torch
    b, n = 16, 128
    mats, truths, gbars, refs = [], [], [], []
    for i in range(b):
        a, q, lam = W.spd_range(n, 1e-2, 1e2, 100 + i)
        mats.append(a)
        truths.append((q * np.sqrt(lam)) @ q.T)
        gb = W.gaussian((n, n), 200 + i)
        gbars.append(gb)
        refs.append(oracle.adjoint_spd(q, lam, gb))
    # row-major batch of symmetric matrices is a valid column-major batch
    a_d = torch.from_numpy(np.ascontiguousarray(np.stack(mats))).cuda()
    x, info, f = msq.sqrtm(a_d, keep_factor=True)
    assert info["relres"] <= 1e-13
    xh = x.cpu().numpy()
    for i in range(b):
        assert oracle.relerr(xh[i], truths[i]) <= 1e-11
    g, binfo = msq.sqrtm_backward(f, x, torch.from_numpy(np.ascontiguousarray(np.stack(gbars))).cuda())
    gh = g.cpu().numpy()
    # row-major gbar = (column-major gbar)^T; the adjoint transposes with it
    for i in range(b):
        assert oracle.relerr(gh[i], refs[i]) <= 1e-10


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("n", [1, 2, 33, 34, 65, 100])
def test_batched_eigensolver_tree_shapes(msq, prec, n):
    # the batch is diagonalised as one block-diagonal tridiagonal matrix:
    # sizes with a single leaf (1, 2), one merge (33 -> 16 + 17; 34 also ends
    # the reduction with a one-column panel), a leaf carried through a level
    # (65 -> 32 | 33) and uneven halves (100)
    import torch
    b = 3
    mats, truths = [], []
    for i in range(b):
        a, q, lam = W.spd_range(n, 1e-2, 1e2, 400 + 10 * n + i)
        mats.append(a)
        truths.append((q * np.sqrt(lam)) @ q.T)
    a_d = torch.from_numpy(np.ascontiguousarray(np.stack(mats))).cuda()
    x, info = msq.sqrtm(a_d, prec=prec, fallback=False)
    assert info["relres"] <= 1e-13
    xh = x.cpu().numpy()
    for i in range(b):
        assert oracle.relerr(xh[i], truths[i]) <= 1e-11


def test_autograd_function(msq):
    import torch
    n = 40
    a, q, lam = W.spd(n, 1e3, 21)
    gbar = W.gaussian((n, n), 22)
    ad = _dev(a).requires_grad_(True)
    x = msq.sqrtm_autograd(ad)
    loss = (x * _dev(gbar)).sum()
    loss.backward()
    ref = oracle.adjoint_spd(q, lam, gbar)
    assert oracle.relerr(ad.grad.cpu().numpy(), ref) <= 1e-10
