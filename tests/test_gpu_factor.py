"""GPU parity of the on-device spectral decomposition (tridiagonalisation,
divide and conquer, back-transformation) and of the full SPD solve
(Alg. 3) through the C-ABI, against the CPU oracle and exact constructions."""

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


def _check_factor(msq, a, prec, tol_scale=1.0):
    n = a.shape[0]
    f = msq.factor(_dev(a), prec=prec)
    q, s, k = f.export(single=(prec == "fp32"))
    q = q[0].astype(np.float64)
    lam = s[0].astype(np.float64) ** 2
    u = 6e-8 if prec == "fp32" else 1.1e-16
    asc = a / 4.0 ** k
    ortho = np.linalg.norm(q.T @ q - np.eye(n))
    back = np.linalg.norm((q * lam) @ q.T - asc) / np.linalg.norm(asc)
    ref = np.linalg.eigvalsh(asc)
    eig_err = np.abs(np.sort(lam) - ref).max() / np.abs(ref).max()
    bound = tol_scale * 50 * max(n, 10) * u
    assert ortho <= bound, (n, prec, ortho, bound)
    assert back <= bound, (n, prec, back, bound)
    assert eig_err <= bound, (n, prec, eig_err, bound)
    assert np.all(np.diff(lam) >= 0)  # ascending
    return q, lam


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("n", [1, 2, 3, 17, 32, 33, 65, 130, 257, 600])
def test_factor_spd(msq, n, prec):
    a, _, _ = W.spd(n, 1e4, 300 + n)
    _check_factor(msq, a, prec)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_factor_deflation_cases(msq, prec):
    # repeated eigenvalues (heavy deflation), a diagonal matrix (zero
    # off-diagonals), the identity, and clustered Hilbert spectrum
    n = 150
    q = W.haar_orthogonal(n, np.random.Generator(np.random.PCG64(5)))
    lam = np.repeat([1.0, 2.0, 3.0], 50)
    a = (q * lam) @ q.T
    a = 0.5 * (a + a.T)
    _check_factor(msq, a, prec)
    _check_factor(msq, np.diag(np.linspace(1.0, 5.0, 77)), prec)
    _check_factor(msq, np.eye(40), prec)
    _check_factor(msq, W.hilbert(120, 1e-3), prec)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("n,kappa", [(1, 1.0), (2, 1e2), (33, 1e4), (256, 1e4), (700, 1e6)])
def test_sqrtm_spd_end_to_end(msq, n, kappa, prec):
    a, q, lam = W.spd(n, kappa, 400 + n)
    x, info = msq.sqrtm(_dev(a), prec=prec, tol=1e-13, fallback=False)
    x = x.cpu().numpy()
    xt = (q * np.sqrt(lam)[None, :]) @ q.T
    assert info["struct_used"] == "hpd"
    assert oracle.relres(x, a) <= 1e-13
    bound = 1e-11 if kappa <= 1e4 else 1e-10
    assert oracle.relerr(x, xt) <= bound
    assert np.array_equal(x, x.T)
    if prec == "fp64":
        assert info["steps"] <= 1
    else:
        assert info["steps"] <= 3 if kappa <= 1e4 else info["steps"] <= 8


def test_sqrtm_matches_oracle_routes(msq):
    n = 300
    a, _, _ = W.spd(n, 1e3, 77)
    x, _ = msq.sqrtm(_dev(a))
    x = x.cpu().numpy()
    assert oracle.relerr(x, oracle.sqrtm_spd(a)) <= 1e-11
    assert oracle.relerr(x, oracle.sqrtm(a)) <= 1e-11


def test_scaling_exponent_is_exact(msq):
    # A and 4^10 A: the root scales by exactly 2^10 (power-of-4 scaling).
    n = 64
    a, _, _ = W.spd(n, 1e2, 5)
    x1, i1 = msq.sqrtm(_dev(a))
    x2, i2 = msq.sqrtm(_dev(a * 4.0 ** 10))
    assert i2["scale_exp"] == i1["scale_exp"] + 10
    assert np.array_equal(x1.cpu().numpy() * 2.0 ** 10, x2.cpu().numpy())


def test_sqrtm_deterministic(msq):
    a, _, _ = W.spd(200, 1e4, 6)
    x1, _ = msq.sqrtm(_dev(a))
    x2, _ = msq.sqrtm(_dev(a))
    import torch
    assert torch.equal(x1, x2)


def test_status_codes(msq):
    import torch
    from paper_2607_12430_amd import MsqrtError
    a = np.eye(8)
    a[3, 3] = np.nan
    with pytest.raises(MsqrtError) as e:
        msq.sqrtm(_dev(a))
    assert e.value.name == "nonfinite"
    # symmetric indefinite: no principal root even in FP64
    b = np.diag([1.0, -1.0, 2.0])
    x, info = msq.sqrtm(_dev(b), allow_fail=True)
    assert info["status"] == "no_principal"
    # maxit = 0 on a FP32 factor leaves X_0 and reports not_converged
    c, _, _ = W.spd(50, 1e4, 3)
    x, info = msq.sqrtm(_dev(c), maxit=0, fallback=False, allow_fail=True)
    assert info["status"] == "not_converged"
    # empty input is fine
    x, info = msq.sqrtm(torch.zeros((0, 0), dtype=torch.float64, device="cuda"))
    assert x.shape == (0, 0)


def test_fallback_to_fp64_when_fp32_sees_nonpositive_eigenvalue(msq):
    # kappa ~ 1e9: float32 eigenvalues of the tiny end can go <= 0
    a = W.hilbert(160, 1e-9)
    x, info = msq.sqrtm(_dev(a), prec="fp32", fallback=True, allow_fail=True)
    if info["status"] == "ok":
        xh = x.cpu().numpy()
        assert oracle.relres(xh, a) <= 1e-13
    assert info["fallbacks"] >= 1 or info["prec_used"] == "fp32"
