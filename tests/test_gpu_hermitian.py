"""Complex Hermitian positive definite input (Alg. 3 with F = C): the solve,
factor + refinement and backward through the C-ABI against the float64 oracle
(complex Schur method), the generator's exact root and Kronecker brute
force.  The library solves it through the real representation
[[Re A, -Im A], [Im A, Re A]], so the checks also cover that the root read
back is exactly Hermitian."""

import time

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


def _elementwise(x, xref):
    return float(np.abs(x - xref).max() / np.abs(xref).max())


def _truth(u, lam):
    return (u * np.sqrt(lam)[None, :]) @ u.conj().T


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("n", [1, 2, 37, 300])
def test_hpd_complex_against_oracle(msq, n, prec):
    a, u, lam = W.hpd(n, 1e4, 800 + n)
    x, info = msq.sqrtm(_dev(a), prec=prec, fallback=False)
    xh = x.cpu().numpy()
    assert info["struct_used"] == "hpd" and info["prec_used"] == prec
    assert info["relres"] <= 1e-13 and oracle.relres(xh, a) <= 1e-13
    assert np.array_equal(xh, xh.conj().T)  # exactly Hermitian
    xo = oracle.sqrtm(a)
    assert oracle.relerr(xh, xo) <= 1e-11 and _elementwise(xh, xo) <= 1e-11
    assert oracle.relerr(xh, _truth(u, lam)) <= 1e-11
    if prec == "fp32" and n > 2:
        assert 1 <= info["steps"] <= 3


def test_hpd_complex_1024_faster_than_general_route(msq):
    """The same Hermitian input through the symmetric route and through the
    general (complex Schur) route: both match the oracle; the symmetric route
    is the faster one."""
    import torch
    n = 1024
    a, u, lam = W.hpd(n, 1e4, 901)
    at = _dev(a)
    times = {}
    res = {}
    for structure in ("auto", "general"):
        msq.sqrtm(at, prec="fp32", structure=structure, fallback=False)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info = msq.sqrtm(at, prec="fp32", structure=structure, fallback=False)
        torch.cuda.synchronize()
        times[structure] = time.perf_counter() - t0
        res[structure] = (x.cpu().numpy(), info)
    print(f"complex HPD n={n}: symmetric route {times['auto'] * 1e3:.1f} ms, "
          f"general route {times['general'] * 1e3:.1f} ms", flush=True)
    assert res["auto"][1]["struct_used"] == "hpd"
    assert res["general"][1]["struct_used"] == "general"
    xo = oracle.sqrtm(a)
    for x, info in res.values():
        assert info["relres"] <= 1e-13
        assert oracle.relerr(x, xo) <= 1e-11 and _elementwise(x, xo) <= 1e-11
    assert times["auto"] < times["general"]


def test_hpd_complex_batch(msq):
    import torch
    b, n = 6, 65
    mats, truths = [], []
    for i in range(b):
        a, u, lam = W.hpd(n, 1e3, 910 + i)
        mats.append(a)
        truths.append(_truth(u, lam))
    # a row-major batch holds the transposes A^T = conj(A), also Hermitian
    ad = torch.from_numpy(np.ascontiguousarray(np.stack(mats))).cuda()
    x, info = msq.sqrtm(ad, prec="fp32", fallback=False)
    assert info["struct_used"] == "hpd" and info["relres"] <= 1e-13
    xh = x.cpu().numpy()
    for i in range(b):
        assert oracle.relerr(xh[i], truths[i]) <= 1e-11
        assert oracle.relerr(xh[i], oracle.sqrtm(mats[i])) <= 1e-11


def test_hpd_complex_factor_then_refine_nearby(msq):
    n = 120
    a, u, lam = W.hpd(n, 1e2, 920)
    z = W.gaussian((2, n, n), 921)
    e = (z[0] + 1j * z[1])
    e = e + e.conj().T
    a2 = a + 1e-6 * e / np.linalg.norm(e)
    f = msq.factor(_dev(a), prec="fp32")
    x0 = _truth(u, lam)
    x0 = 0.5 * (x0 + x0.conj().T)
    xd = _dev(x0)
    info = msq.refine(f, _dev(a2), xd, init_from_factor=False)
    x = xd.cpu().numpy()
    assert info["status"] == "ok" and info["steps"] >= 1
    assert oracle.relres(x, a2) <= 1e-13
    assert oracle.relerr(x, oracle.sqrtm(a2)) <= 1e-11
    xd = _dev(np.zeros((n, n), np.complex128))
    info = msq.refine(f, _dev(a), xd, init_from_factor=True)
    assert info["status"] == "ok" and oracle.relerr(xd.cpu().numpy(), _truth(u, lam)) <= 1e-11


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("n", [5, 48])
def test_hpd_complex_backward_against_oracle(msq, n, prec):
    """X^H G + G X^H = Gbar (X Hermitian: X G + G X = Gbar) against the
    oracle's Schur-form adjoint and, for n <= 8, the Kronecker system."""
    a, u, lam = W.hpd(n, 1e3, 930 + n)
    g0 = W.gaussian((2, n, n), 931 + n)
    gbar = g0[0] + 1j * g0[1]
    x, info, f = msq.sqrtm(_dev(a), prec=prec, keep_factor=True, fallback=False)
    g, binfo = msq.sqrtm_backward(f, x, _dev(gbar))
    g = g.cpu().numpy()
    xh = x.cpu().numpy()
    assert binfo["relres"] <= 1e-13
    assert oracle.relerr(g, oracle.adjoint(xh, gbar)) <= 1e-10
    if n <= 8:
        assert oracle.relerr(g, oracle.kron_adjoint(xh, gbar)) <= 1e-10


def test_hpd_complex_structure_errors(msq):
    n = 40
    a, _, _ = W.hpd(n, 1e2, 940)
    bad = a.copy()
    bad[3, 17] += 1e-3j  # no longer Hermitian
    _, info = msq.sqrtm(_dev(bad), structure="hpd", allow_fail=True)
    assert info["status"] == "invalid_arg"
    x, info = msq.sqrtm(_dev(bad), prec="fp32")  # AUTO: general path
    assert info["struct_used"] == "general"
    assert oracle.relerr(x.cpu().numpy(), oracle.sqrtm(bad)) <= 1e-11
    # Hermitian but indefinite: no principal root, confirmed in FP64
    u = W.haar_unitary(n, np.random.default_rng(941))
    lam = np.linspace(-1.0, 2.0, n)
    ind = (u * lam) @ u.conj().T
    ind = 0.5 * (ind + ind.conj().T)
    _, info = msq.sqrtm(_dev(ind), prec="fp32", allow_fail=True)
    assert info["status"] == "no_principal"
