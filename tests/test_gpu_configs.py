"""The workload configurations at their full sizes, in the launch
configuration the benchmark uses (msqrt_sqrtm with A resident on the device):

* C1  SPD n=256, eigenvalues log-uniform on [1e-2, 1e2], float64 factor;
* C2s SPD n=4096, kappa in {1e2, 1e4, 1e6}, float32 factor (seeds 2, 3, 4);
* C5  64 SPD matrices n=512 (eigenvalues log-uniform on [1e-2, 1e2]) solved
      as one batch, forward and backward, with central differences;
* C2n real nonsymmetric n=2048, A = 2 I + G / sqrt(n) (seed 5);
* C3  the complex A = B^2 family at n=1024 and at its full size n=8192
      (host-side generation about 25 s, solve about 21 s on one MI355X).

Expected values: the generator's exact roots (X = Q diag(lam^1/2) Q^T for SPD
inputs, X = B for A = B^2), the oracle where it finishes in seconds, and
otherwise properties that hold at any size (residual, commutation with A,
principal spectrum)."""

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


def _msq():
    import paper_2607_12430_amd as msq
    return msq


def _t(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _relres_gpu(x, a):
    import torch
    return float(torch.linalg.matrix_norm(x @ x - a) / torch.linalg.matrix_norm(a))


def test_c1_spd_256_fp64_factor():
    msq = _msq()
    a, q, lam = W.spd_range(256, 1e-2, 1e2, 1)
    x_true = (q * np.sqrt(lam)) @ q.T
    x, info = msq.sqrtm(_t(a), prec="fp64", fallback=False)
    xh = x.cpu().numpy()
    assert info["prec_used"] == "fp64" and info["struct_used"] == "hpd"
    assert info["relres"] <= 1e-13
    assert oracle.relres(xh, a) <= 1e-13
    assert oracle.relerr(xh, x_true) <= 1e-11
    assert oracle.relerr(xh, oracle.sqrtm_spd(a)) <= 1e-11
    assert oracle.relerr(xh, oracle.sqrtm(a)) <= 1e-11


@pytest.mark.parametrize("kappa,seed,tol", [(1e2, 2, 1e-11), (1e4, 3, 1e-11), (1e6, 4, 1e-10)])
def test_c2s_spd_4096(kappa, seed, tol):
    msq = _msq()
    a, q, lam = W.spd(4096, kappa, seed)
    x_true = (q * np.sqrt(lam)) @ q.T
    at = _t(a)
    x, info = msq.sqrtm(at, prec="fp32", fallback=False)
    assert info["prec_used"] == "fp32"
    assert info["relres"] <= 1e-13
    assert _relres_gpu(x, at) <= 1e-13
    assert 1 <= info["steps"] <= 4
    assert oracle.relerr(x.cpu().numpy(), x_true) <= tol


def test_c5_batched_forward_backward_with_finite_differences():
    import torch
    msq = _msq()
    n, b = 512, 64
    mats, qs, lams, gbars = [], [], [], []
    for i in range(b):
        a, q, lam = W.spd_range(n, 1e-2, 1e2, 100 + i)
        mats.append(a)
        qs.append(q)
        lams.append(lam)
        gbars.append(W.gaussian((n, n), 200 + i))
    a_d = torch.from_numpy(np.ascontiguousarray(np.stack(mats))).cuda()
    x, info, f = msq.sqrtm(a_d, prec="fp32", keep_factor=True, fallback=False)
    assert info["relres"] <= 1e-13
    xh = x.cpu().numpy()
    for i in range(b):
        x_true = (qs[i] * np.sqrt(lams[i])) @ qs[i].T
        assert oracle.relerr(xh[i], x_true) <= 1e-11
    g_d = torch.from_numpy(np.ascontiguousarray(np.stack(gbars))).cuda()
    g, binfo = msq.sqrtm_backward(f, x, g_d)
    assert binfo["relres"] <= 1e-13
    gh = g.cpu().numpy()
    for i in range(b):
        # the library sees each row-major buffer as its transpose; for
        # symmetric A and X the adjoint of Gbar^T is G^T
        g_ref = oracle.adjoint_spd(qs[i], lams[i], gbars[i].T).T
        assert oracle.relerr(gh[i], g_ref) <= 1e-10
    # central differences of f(A) = <Gbar, sqrtm(A)> along symmetric unit
    # directions, h = 1e-6, for two matrices of the batch
    h = 1e-6
    for i in (0, 37):
        for d in range(2):
            z = W.gaussian((n, n), 300 + 2 * i + d)
            e = z + z.T
            e /= np.linalg.norm(e)
            fp, fm = [], []
            for sgn, store in ((1.0, fp), (-1.0, fm)):
                xs, _ = msq.sqrtm(_t(mats[i] + sgn * h * e), prec="fp32", tol=1e-14,
                                  fallback=False)
                store.append(float(np.sum(gbars[i] * xs.cpu().numpy())))
            fd = (fp[0] - fm[0]) / (2 * h)
            an = float(np.sum(gh[i] * e))
            # relative to ||G||_F, the largest <G, E> over unit directions
            assert abs(fd - an) <= 1e-6 * np.linalg.norm(gh[i])


def test_c2n_real_nonsymmetric_2048():
    msq = _msq()
    a = W.nonsym_shifted(2048, 5)
    at = _t(a)
    x, info = msq.sqrtm(at, prec="fp32", fallback=False)
    assert info["struct_used"] == "general"
    assert info["relres"] <= 1e-13
    assert _relres_gpu(x, at) <= 1e-13
    xh = x.cpu().numpy()
    comm = np.linalg.norm(xh @ a - a @ xh) / (np.linalg.norm(xh) * np.linalg.norm(a))
    assert comm <= 1e-13
    # principal: every eigenvalue of X in the open right half-plane, and they
    # are the square roots of the eigenvalues of A
    ev = np.linalg.eigvals(xh)
    assert np.all(ev.real > 0)
    lam = np.linalg.eigvals(a)
    from scipy.optimize import linear_sum_assignment
    cost = np.abs(np.sqrt(lam)[:, None] - ev[None, :])
    r, c = linear_sum_assignment(cost)
    assert np.max(cost[r, c]) <= 1e-8


def test_c3_complex_square_family_1024():
    msq = _msq()
    a, bmat = W.complex_square(1024, 6)
    at = _t(a)
    x, info = msq.sqrtm(at, prec="fp32", fallback=False)
    assert info["relres"] <= 1e-13
    assert _relres_gpu(x, at) <= 1e-13
    assert oracle.relerr(x.cpu().numpy(), bmat) <= 1e-10


def test_c3_complex_square_8192_full_size():
    """Full-size C3: complex128 A = B^2, n = 8192, complex64 Schur factor,
    complex128 refinement.  Checked on the GPU against the generator's exact
    root B and by properties that hold at any size (residual, commutation
    with A)."""
    import time
    import torch
    msq = _msq()
    n = 8192
    a, bmat = W.complex_square(n, 6)
    at, bt = _t(a), _t(bmat)
    del a, bmat
    t0 = time.perf_counter()
    x, info = msq.sqrtm(at, prec="fp32", fallback=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(f"C3 n={n}: {dt:.2f} s, steps {info['steps']}, relres {info['relres']:.2e}, "
          f"phases {info['t_ms']}", flush=True)
    assert info["prec_used"] == "fp32" and info["struct_used"] == "general"
    assert info["relres"] <= 1e-13
    assert _relres_gpu(x, at) <= 1e-13
    assert float(torch.linalg.matrix_norm(x - bt) / torch.linalg.matrix_norm(bt)) <= 1e-10
    comm = torch.linalg.matrix_norm(x @ at - at @ x) / (torch.linalg.matrix_norm(x) *
                                                        torch.linalg.matrix_norm(at))
    assert float(comm) <= 1e-13
