"""Pins of the oracle's real quasi-triangular route (remark in Sec. 2.2.1:
real Schur form A = Q T Q^T with 1x1 and 2x2 diagonal blocks, no 2x2 block
cut by a block partition).  Each check compares against something other than
the routine itself: the eigendecomposition of a 2x2 block, a quasi-triangular
matrix built as the square of a known root, the Kronecker form of the
Sylvester equation, the oracle's independent complex Schur route and
scipy's sqrtm."""

import numpy as np
import pytest
import scipy.linalg

import oracle as O


def _quasi(rng, n, pairs, alpha_lo=0.5, upper=0.3):
    """Quasi-upper-triangular U of order n whose 2x2 blocks start at the
    indices in `pairs`: block [[a, b], [c, a]] with a > 0 and b c < 0
    (eigenvalues a +- i sqrt(-b c), in the right half-plane); 1x1 blocks are
    positive.  The strictly upper part is random."""
    u = np.triu(rng.standard_normal((n, n)) * upper, 1)
    i = 0
    while i < n:
        if i in pairs:
            a = rng.uniform(alpha_lo, 2.0)
            b = rng.uniform(0.3, 1.5) * rng.choice([-1.0, 1.0])
            c = -np.sign(b) * rng.uniform(0.3, 1.5)
            u[i, i] = u[i + 1, i + 1] = a
            u[i, i + 1] = b
            u[i + 1, i] = c
            i += 2
        else:
            u[i, i] = rng.uniform(alpha_lo, 2.0)
            i += 1
    return u


def test_sqrt_2x2_matches_eigendecomposition():
    rng = np.random.default_rng(3)
    for _ in range(50):
        b = rng.standard_normal((2, 2))
        lam, v = np.linalg.eig(b)
        if np.any((np.abs(lam.imag) < 1e-12) & (lam.real <= 0)):
            continue
        ref = (v @ np.diag(np.sqrt(lam.astype(complex))) @ np.linalg.inv(v)).real
        x = O.sqrt_2x2(b)
        assert np.allclose(x, ref, rtol=1e-12, atol=1e-12)
        assert np.linalg.norm(x @ x - b) <= 1e-14 * max(1.0, np.linalg.norm(b))
    # a block with a real negative eigenvalue has no real principal root
    with pytest.raises(O.OracleError):
        O.sqrt_2x2(np.array([[-1.0, 0.5], [0.2, 2.0]]))


@pytest.mark.parametrize("single", [False, True])
def test_trsqrt_quasi_recovers_known_root(single):
    rng = np.random.default_rng(5)
    n = 41
    u = _quasi(rng, n, pairs={0, 5, 7, 19, 30, 39})
    t = u @ u
    # T keeps U's block structure: the same nonzero subdiagonal entries
    assert np.allclose(np.tril(t, -2), 0)
    assert np.array_equal(np.abs(np.diag(t, -1)) > 0, np.abs(np.diag(u, -1)) > 0)
    got = O.trsqrt_quasi(t, single=single)
    err = np.linalg.norm(got - u) / np.linalg.norm(u)
    assert err <= (2e-5 if single else 1e-13), err


def test_trsqrt_quasi_negative_real_eigenvalue_has_no_principal_root():
    rng = np.random.default_rng(6)
    u = _quasi(rng, 9, pairs={2})
    t = u @ u
    t[6, 6] = -abs(t[6, 6])
    with pytest.raises(O.OracleError):
        O.trsqrt_quasi(t)


@pytest.mark.parametrize("m,n", [(11, 4), (4, 11), (11, 10), (12, 12)])
def test_rtrsyl_quasi_matches_kronecker_every_branch(m, n):
    """Rows-only (2n <= m), columns-only (2m <= n) and the four-block branch
    of Alg. 1, with a 2x2 block straddling every natural split point
    floor(m/2), so that a split which cut it would drop the coupling entry
    and fail."""
    rng = np.random.default_rng(7 + m + 3 * n)

    def straddling(k):
        h = k // 2
        pairs = {h - 1}
        if k >= 8:
            pairs.add(h // 2 - 1 if (h // 2 - 1) not in (h - 2, h) else 0)
        return _quasi(rng, k, pairs=pairs)

    s, st = straddling(m), straddling(n)
    assert s[m // 2, m // 2 - 1] != 0 and st[n // 2, n // 2 - 1] != 0
    c = rng.standard_normal((m, n))
    ref = O.kron_sylvester(s, st, c).real
    for blks in (1, 2, 3):
        y = O.rtrsyl_quasi(s, st, c, blks=blks)
        assert np.linalg.norm(y - ref) <= 1e-13 * np.linalg.norm(ref)
    y = O.trsyl_quasi(s, st, c)
    assert np.linalg.norm(y - ref) <= 1e-13 * np.linalg.norm(ref)
    ys = O.rtrsyl_quasi(s, st, c, blks=2, single=True)
    assert np.linalg.norm(ys - ref) <= 1e-5 * np.linalg.norm(ref)


@pytest.mark.parametrize("n,seed", [(40, 1), (64, 2), (97, 3)])
def test_sqrtm_real_agrees_with_complex_route_and_scipy(n, seed):
    rng = np.random.default_rng(seed)
    a = 2.0 * np.eye(n) + rng.standard_normal((n, n)) / np.sqrt(n)
    x, fac = O.sqrtm_real(a, return_factors=True)
    t = fac["T"]
    assert np.sum(np.abs(np.diag(t, -1)) > 0) >= 4  # complex pairs present
    assert np.linalg.norm(fac["Q"] @ t @ fac["Q"].T - a) <= 1e-13 * np.linalg.norm(a)
    assert O.relerr(x, O.sqrtm(a)) <= 1e-12
    assert O.relerr(x, scipy.linalg.sqrtm(a).real) <= 1e-12
    assert O.relres(x, a) <= 1e-13


def test_emulator_real_route_converges_to_the_root():
    rng = np.random.default_rng(11)
    n = 128
    a = 2.0 * np.eye(n) + rng.standard_normal((n, n)) / np.sqrt(n)
    xr = O.sqrtm_real(a)
    real = O.emulate_mixed(a, structure="general", schur_form="real")
    cplx = O.emulate_mixed(a, structure="general")
    assert real["status"] == "ok" and cplx["status"] == "ok"
    assert O.relerr(real["X"], xr) <= 1e-12
    # the first residual is that of the float32 factor (unit roundoff level)
    assert 1e-8 < real["hist"][0] < 1e-5
    assert abs(real["steps"] - cplx["steps"]) <= 1
    null = O.emulate_mixed(a, structure="general", schur_form="real", tol=-1.0, maxit=4)
    assert null["status"] == "ok" and null["steps"] == 4 and len(null["hist"]) == 5
    # a real negative eigenvalue: no principal root with the float factor
    b = a.copy()
    b[0, :] = 0.0
    b[:, 0] = 0.0
    b[0, 0] = -1.0
    assert O.emulate_mixed(b, structure="general", schur_form="real")["status"] == "no_principal"
