"""The device-side input generators (run here on the CPU device): the laws
they implement, pinned by their defining properties."""

import numpy as np
import pytest

import workloads as W


@pytest.fixture(scope="module")
def D():
    import workloads.device as d
    return d


def test_haar_orthogonal_is_orthogonal(D):
    import torch
    q = D.haar_orthogonal(50, D._gen(3, "cpu"), "cpu").numpy()
    assert np.linalg.norm(q.T @ q - np.eye(50)) <= 1e-13


@pytest.mark.parametrize("n,kappa", [(1, 10.0), (2, 1e3), (40, 1e6), (200, 1e2)])
def test_spd_condition_number_is_exact(D, n, kappa):
    a = D.spd(n, kappa, 7, "cpu").numpy()
    assert np.array_equal(a, a.T)
    lam = np.linalg.eigvalsh(a)
    if n == 1:
        assert abs(lam[0] - 1.0) <= 1e-15
        return
    assert abs(lam[0] - kappa ** -0.5) <= 1e-10 * kappa ** 0.5
    assert abs(lam[-1] - kappa ** 0.5) <= 1e-10 * kappa ** 0.5
    assert lam.min() > 0


def test_nonsym_shifted_law(D):
    n = 300
    a = D.nonsym_shifted(n, 11, "cpu").numpy()
    g = (a - 2.0 * np.eye(n)) * np.sqrt(n)
    # i.i.d. N(0, 1) entries: sample mean and variance
    assert abs(g.mean()) <= 5.0 / n
    assert abs(g.var() - 1.0) <= 0.02


def test_nonsym_kappa_spectrum(D):
    n, kappa = 60, 1e4
    a = D.nonsym_kappa(n, kappa, 5, "cpu").numpy()
    ev = np.sort(np.linalg.eigvals(a).real)
    # the eigenvalues are those of the diagonal part: log-uniform with pinned ends
    assert abs(ev[0] - kappa ** -0.5) <= 1e-8
    assert abs(ev[-1] - kappa ** 0.5) <= 1e-8 * kappa ** 0.5
    assert not np.allclose(a, a.T)


def test_selector_params_match_host(D):
    for idx in (0, 1, 17, 10_001, 50_123):
        _, kind, n, kappa = W.selector_matrix(idx, 320)
        k2, n2, kap2, _ = W.selector_params(idx, 320)
        assert (kind, n, kappa) == (k2, n2, kap2)
        a, k3, n3, kap3 = D.selector_matrix(idx, 320, "cpu")
        assert (k3, n3, kap3) == (kind, n, kappa) and tuple(a.shape) == (n, n)
