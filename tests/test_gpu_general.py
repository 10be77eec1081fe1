"""General path (Alg. 2) on the GPU against the oracle: Hessenberg reduction,
complex Schur QR, triangular square root, triangular Sylvester solver, the
complete solve for real nonsymmetric and complex input, and the backward
solve.  Results that are not unique (the Hessenberg form, the Schur vectors)
are checked through what is unique (eigenvalues, the reconstructed matrix)
and the defining properties (unitarity, triangular structure)."""

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
U64 = 2.0 ** -53


def _msq():
    import paper_2607_12430_amd as msq
    return msq


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _unit_err(q):
    n = q.shape[0]
    return float(np.linalg.norm(q.conj().T @ q - np.eye(n)))


def _match_eigs(a, b):
    from scipy.optimize import linear_sum_assignment
    cost = np.abs(a[:, None] - b[None, :])
    r, c = linear_sum_assignment(cost)
    return float(np.max(cost[r, c]))


def _complex_input(n, seed):
    a, _ = W.complex_square(n, seed)
    return np.asfortranarray(a)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("n", [1, 2, 3, 5, 33, 64, 100, 130])
def test_gehrd_properties(prec, n):
    msq = _msq()
    a = _complex_input(n, 11 + n)
    h, q = msq.test_gehrd(a, prec=prec)
    u = U32 if prec == "fp32" else U64
    assert np.all(np.tril(h, -2) == 0)
    assert _unit_err(q) <= 20 * np.sqrt(n) * u * np.sqrt(n)
    assert _rel(q @ h @ q.conj().T, a) <= 20 * np.sqrt(n) * u


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("n,kind", [(1, "c"), (2, "c"), (3, "r"), (17, "c"), (64, "r"), (96, "c"),
                                    (97, "r"), (130, "c"), (200, "r"), (300, "c")])
def test_schur_against_oracle(prec, n, kind):
    msq = _msq()
    a = _complex_input(n, 21 + n) if kind == "c" else W.nonsym_shifted(n, 21 + n).astype(np.complex128)
    a = np.asfortranarray(a)
    t, q = msq.test_schur(a, prec=prec)
    u = U32 if prec == "fp32" else U64
    assert np.all(np.tril(t, -1) == 0)
    # backward-stable QR: O(n u) unitarity and reconstruction errors
    assert _unit_err(q) <= 50 * n * u
    assert _rel(q @ t @ q.conj().T, a) <= 20 * n * u
    t_ref, _ = oracle.schur(a)
    lam_ref = np.diag(t_ref)
    # eigenvalues agree to the backward error times a modest condition factor
    err = _match_eigs(np.diag(t), lam_ref)
    assert err <= 1e4 * np.sqrt(n) * u * np.max(np.abs(lam_ref))


def _schur_root_pair(n, seed):
    a = _complex_input(n, seed)
    t, _ = oracle.schur(a)
    return np.asfortranarray(t)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("n", [1, 5, 32, 33, 64, 100, 200])
def test_trsqrt_against_oracle(prec, n):
    msq = _msq()
    t = _schur_root_pair(n, 31 + n)
    s = msq.test_trsqrt(t, prec=prec)
    s_ref = oracle.trsqrt(t)
    assert np.all(np.tril(s, -1) == 0)
    tol = 2e-5 if prec == "fp32" else 1e-12
    assert _rel(s, s_ref) <= tol
    assert np.all(np.diag(s).real > 0)


def test_trsqrt_negative_eigenvalue_is_rejected():
    msq = _msq()
    t = np.triu(np.ones((40, 40), np.complex128)) + np.eye(40)
    t[17, 17] = -3.0
    with pytest.raises(msq.MsqrtError) as e:
        msq.test_trsqrt(t, prec="fp32")
    assert e.value.name == "no_principal"


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("m,p", [(1, 1), (5, 7), (32, 32), (33, 65), (100, 40), (130, 130)])
def test_trsyl_against_oracle(prec, m, p):
    msq = _msq()
    s = oracle.trsqrt(_schur_root_pair(m, 41 + m))
    s2 = oracle.trsqrt(_schur_root_pair(p, 43 + p))
    rng = np.random.Generator(np.random.PCG64(45 + m + p))
    c = rng.standard_normal((m, p)) + 1j * rng.standard_normal((m, p))
    y = msq.test_trsyl(s, s2, c, prec=prec)
    y_ref = oracle.trsyl(s, s2, c)
    tol = 2e-5 if prec == "fp32" else 1e-12
    assert _rel(y, y_ref) <= tol
    if m * p <= 144:
        assert _rel(y, oracle.kron_sylvester(s, s2, c)) <= max(tol, 1e-11)


def _torch():
    import torch
    return torch


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("n", [1, 8, 100, 257])
def test_sqrtm_real_nonsymmetric(prec, n):
    torch = _torch()
    msq = _msq()
    a = W.nonsym_shifted(n, 51 + n)
    x, info = msq.sqrtm(torch.from_numpy(np.ascontiguousarray(a)).cuda(), prec=prec, tol=1e-13,
                        fallback=False)
    x = x.cpu().numpy()
    # a 1 x 1 matrix is symmetric, so AUTO takes the SPD route there
    assert info["struct_used"] == ("hpd" if n == 1 else "general")
    assert info["relres"] <= 1e-13
    assert oracle.relres(x, a) <= 1e-13
    assert oracle.relerr(x, oracle.sqrtm(a)) <= 1e-11


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("n", [1, 9, 96, 97, 200])
def test_sqrtm_complex(prec, n):
    torch = _torch()
    msq = _msq()
    a, b = W.complex_square(n, 61 + n)
    x, info = msq.sqrtm(torch.from_numpy(np.ascontiguousarray(a)).cuda(), prec=prec, tol=1e-13,
                        fallback=False)
    x = x.cpu().numpy()
    assert info["relres"] <= 1e-13
    x_ref = oracle.sqrtm(a)
    assert oracle.relerr(x, x_ref) <= 1e-11
    assert oracle.relerr(x, b) <= 1e-10


def test_sqrtm_general_refinement_steps_fp32():
    """The FP32 factor needs a few corrections; the FP64 factor at most one."""
    torch = _torch()
    msq = _msq()
    a = W.nonsym_shifted(300, 71)
    at = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    _, i32 = msq.sqrtm(at, prec="fp32", fallback=False)
    _, i64 = msq.sqrtm(at, prec="fp64", fallback=False)
    assert 1 <= i32["steps"] <= 4
    assert i64["steps"] <= 1
    hist = i32["relres_hist"]
    assert all(hist[k + 1] < hist[k] for k in range(len(hist) - 1))


def test_general_no_principal_root():
    torch = _torch()
    msq = _msq()
    rng = np.random.Generator(np.random.PCG64(81))
    n = 40
    v = rng.standard_normal((n, n)) + 4 * np.eye(n)
    lam = np.linspace(1.0, 3.0, n)
    lam[7] = -2.0
    a = v @ np.diag(lam) @ np.linalg.inv(v)
    x, info = msq.sqrtm(torch.from_numpy(np.ascontiguousarray(a)).cuda(), prec="fp32",
                        allow_fail=True)
    assert info["status"] == "no_principal"


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("kind,n", [("r", 6), ("r", 70), ("c", 5), ("c", 66)])
def test_backward_general_against_oracle(prec, kind, n):
    torch = _torch()
    msq = _msq()
    if kind == "r":
        a = W.nonsym_shifted(n, 91 + n)
        gbar = W.gaussian((n, n), 92 + n)
    else:
        a, _ = W.complex_square(n, 93 + n)
        g0 = W.gaussian((2, n, n), 94 + n)
        gbar = g0[0] + 1j * g0[1]
    at = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    x, info, f = msq.sqrtm(at, prec=prec, keep_factor=True, fallback=False)
    g, binfo = msq.sqrtm_backward(f, x, torch.from_numpy(np.ascontiguousarray(gbar)).cuda())
    g = g.cpu().numpy()
    xh = x.cpu().numpy()
    # the library sees row-major buffers as transposes; both sides of the
    # adjoint equation transpose consistently, so G is compared directly
    g_ref = oracle.adjoint(xh, gbar)
    assert binfo["relres"] <= 1e-13
    assert oracle.relerr(g, g_ref) <= 1e-10
    if n <= 8:
        assert oracle.relerr(g, oracle.kron_adjoint(xh, gbar)) <= 1e-10
