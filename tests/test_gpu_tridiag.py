"""GPU stage tests of the spectral decomposition: the tridiagonalisation and
the divide-and-conquer eigensolver in isolation (test hooks in
include/msqrt_testing.h), against library eigenvalues and invariants."""

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def msq():
    import paper_2607_12430_amd as m
    return m


def _tri(d, e):
    return np.diag(d) + np.diag(e, 1) + np.diag(e, -1)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n", [2, 5, 33, 34, 64, 65, 97, 129, 130, 200, 300, 1000, 2000])
def test_sytrd_preserves_spectrum(msq, n, prec):
    a, _, lam = W.spd(n, 1e4, 500 + n)
    d, e, tau = msq.test_sytrd(a, prec)
    u = 6e-8 if prec == "fp32" else 1.1e-16
    ev = np.linalg.eigvalsh(_tri(d.astype(np.float64), e.astype(np.float64)))
    err = np.abs(ev - np.sort(lam)).max() / lam.max()
    assert err <= 20 * n * u, (n, prec, err)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n", [1, 2, 31, 32, 33, 65, 100, 129, 130, 257, 1000])
def test_stedc_random_tridiagonal(msq, n, prec):
    r = np.random.default_rng(n)
    d = r.standard_normal(n)
    e = r.standard_normal(max(n - 1, 0))
    lam, z = msq.test_stedc(d, e, prec)
    t = _tri(d, e) if n > 1 else np.diag(d)
    u = 6e-8 if prec == "fp32" else 1.1e-16
    ref = np.linalg.eigvalsh(t)
    nt = np.abs(ref).max()
    assert np.abs(lam - ref).max() <= 50 * n * 1.1e-16 * nt + (20 * n * u * nt if prec == "fp32" else 0)
    z = z.astype(np.float64)
    assert np.linalg.norm(z.T @ z - np.eye(n)) <= 50 * n * u
    assert np.linalg.norm(t @ z - z * lam) <= 50 * n * u * nt


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_stedc_deflation(msq, prec):
    # zero couplings, repeated diagonal, glued Wilkinson-like blocks
    n = 200
    d = np.repeat([1.0, 2.0, 3.0, 4.0], 50)
    e = np.zeros(n - 1)
    e[::7] = 1e-3
    lam, z = msq.test_stedc(d, e, prec)
    t = _tri(d, e)
    u = 6e-8 if prec == "fp32" else 1.1e-16
    assert np.abs(lam - np.linalg.eigvalsh(t)).max() <= 100 * n * u * 4
    z = z.astype(np.float64)
    assert np.linalg.norm(z.T @ z - np.eye(n)) <= 100 * n * u


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 9, 10, 16, 17, 18, 19, 31, 33, 64, 100, 257, 300, 1000])
def test_sy2tr_decomposition(msq, n, prec):
    """Two-stage reduction: T has the spectrum of A, Q is orthogonal and
    A = Q T Q^T (n spans one band, a ragged last panel and several panels of
    both band widths, 16 for float and 8 for double)."""
    a, _, lam = W.spd(n, 1e4, 700 + n)
    d, e, q = msq.test_sy2tr(a, prec)
    u = 6e-8 if prec == "fp32" else 1.1e-16
    t = _tri(d.astype(np.float64), e.astype(np.float64))
    q = q.astype(np.float64)
    ev = np.linalg.eigvalsh(t)
    assert np.abs(ev - np.sort(lam)).max() / lam.max() <= 20 * n * u
    assert np.linalg.norm(q.T @ q - np.eye(n)) <= 20 * n * u
    assert np.linalg.norm(q @ t @ q.T - a) / np.linalg.norm(a) <= 20 * n * u


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_sy2tr_structured_inputs(msq, prec):
    """Already tridiagonal, diagonal and block-diagonal inputs: zero columns
    give identity reflectors (tau = 0) at every stage."""
    n = 120
    u = 6e-8 if prec == "fp32" else 1.1e-16
    r = np.random.default_rng(3)
    cases = [np.diag(r.standard_normal(n)),
             _tri(r.standard_normal(n), r.standard_normal(n - 1))]
    blk = np.zeros((n, n))
    for s in range(0, n, 40):
        g = r.standard_normal((40, 40))
        blk[s:s + 40, s:s + 40] = g + g.T
    cases.append(blk)
    for a in cases:
        d, e, q = msq.test_sy2tr(a, prec)
        t = _tri(d.astype(np.float64), e.astype(np.float64))
        q = q.astype(np.float64)
        na = np.linalg.norm(a)
        assert np.abs(np.linalg.eigvalsh(t) - np.linalg.eigvalsh(a)).max() <= 20 * n * u * na
        assert np.linalg.norm(q.T @ q - np.eye(n)) <= 20 * n * u
        assert np.linalg.norm(q @ t @ q.T - a) <= 20 * n * u * na
