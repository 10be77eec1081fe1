"""Pins for the CPU oracle: each test checks the oracle against something other
than itself -- closed forms, exact constructions, invariants, an independent
library routine, multiprecision arithmetic or Kronecker brute force."""

import json
import os

import numpy as np
import pytest

import oracle
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rng(seed):
    return np.random.default_rng(seed)


# ---------------------------------------------------------------------------
# Closed forms


def test_diagonal_principal_branch():
    # Diagonal A: X = diag(sqrt(a_ii)), principal branch (Sec. 1 definition).
    d = np.array([4.0, 0.25, 2.0 + 0j, -3.0 + 1e-3j, -3.0 - 1e-3j, 1j, -1j, 1e-8])
    x = oracle.sqrtm(np.diag(d))
    expect = np.sqrt(d.astype(np.complex128))  # numpy's principal complex sqrt
    assert np.allclose(np.diag(x), expect, rtol=1e-14, atol=0)
    assert np.all(np.diag(x).real > 0)
    assert np.abs(x - np.diag(np.diag(x))).max() == 0


def test_2x2_cayley_hamilton():
    # For 2x2 A with eigenvalues l1, l2 (no eigenvalue on R<=0):
    # sqrt(A) = (A + s I) / t with s = sqrt(l1) sqrt(l2), t = sqrt(l1) + sqrt(l2).
    r = rng(1)
    for _ in range(20):
        a = r.standard_normal((2, 2)) + 1j * r.standard_normal((2, 2)) + 3 * np.eye(2)
        l = np.linalg.eigvals(a)
        sq = np.sqrt(l)
        s = sq[0] * sq[1]
        t = sq[0] + sq[1]
        expect = (a + s * np.eye(2)) / t
        x = oracle.sqrtm(a)
        assert np.abs(x - expect).max() <= 1e-13 * np.abs(expect).max()


def test_upper_triangular_2x2_recurrence():
    # [[a, b], [0, c]] -> [[sqrt a, b/(sqrt a + sqrt c)], [0, sqrt c]] (Eq. (subst), n=2).
    a, b, c = 2.0 + 1j, -0.5 + 3j, 0.3 - 0.1j
    t = np.array([[a, b], [0, c]])
    s = oracle.trsqrt(t)
    sa, sc = np.sqrt(a), np.sqrt(c)
    expect = np.array([[sa, b / (sa + sc)], [0, sc]])
    assert np.abs(s - expect).max() <= 1e-15 * 4


def test_triangular_3x3_hand_expansion():
    # n = 3: s_13 = (t_13 - s_12 s_23) / (s_11 + s_33), written out by hand.
    t = np.array([[4.0, 1.0, 2.0], [0, 9.0, -1.0], [0, 0, 1.0]], dtype=complex)
    s11, s22, s33 = 2.0, 3.0, 1.0
    s12 = 1.0 / (s11 + s22)
    s23 = -1.0 / (s22 + s33)
    s13 = (2.0 - s12 * s23) / (s11 + s33)
    expect = np.array([[s11, s12, s13], [0, s22, s23], [0, 0, s33]])
    s = oracle.trsqrt(t)
    assert np.abs(s - expect).max() <= 1e-15 * 8
    assert np.abs(s @ s - t).max() <= 1e-14


def test_no_principal_root_rejected():
    with pytest.raises(oracle.OracleError):
        oracle.sqrtm(np.diag([1.0, -2.0, 3.0]))
    with pytest.raises(oracle.OracleError):
        oracle.sqrtm(np.diag([1.0, 0.0]))


# ---------------------------------------------------------------------------
# Exact constructions A = B^2


@pytest.mark.parametrize("n,seed", [(8, 6), (40, 7), (96, 8)])
def test_complex_square_known_root(n, seed):
    a, b = W.complex_square(n, seed)
    x = oracle.sqrtm(a)
    assert oracle.relerr(x, b) < 1e-12
    assert oracle.relres(x, a) < 1e-13


@pytest.mark.parametrize("n,kappa,seed", [(16, 1e2, 1), (64, 1e4, 2), (128, 1e6, 3)])
def test_spd_known_root_both_routes(n, kappa, seed):
    a, q, lam = W.spd(n, kappa, seed)
    xt = (q * np.sqrt(lam)[None, :]) @ q.T
    x1 = oracle.sqrtm(a)
    x2 = oracle.sqrtm_spd(a)
    bound = 1e-15 * np.sqrt(kappa) * n * 4
    assert oracle.relerr(x1, xt) < bound
    assert oracle.relerr(x2, xt) < bound
    # the two independent routes agree
    assert oracle.relerr(x1, x2) < bound


# ---------------------------------------------------------------------------
# Factorisations against library routines and invariants


@pytest.mark.parametrize("n", [1, 2, 3, 17, 64])
def test_schur_invariants(n):
    r = rng(n)
    a = r.standard_normal((n, n)) + 1j * r.standard_normal((n, n))
    t, q = oracle.schur(a)
    assert np.abs(np.tril(t, -1)).max(initial=0) == 0
    assert np.linalg.norm(q.conj().T @ q - np.eye(n)) < 1e-13 * max(n, 1)
    assert np.linalg.norm(q @ t @ q.conj().T - a) < 1e-13 * np.linalg.norm(a)
    ev = np.sort_complex(np.diag(t))
    ref = np.sort_complex(np.linalg.eigvals(a))
    assert np.abs(ev - ref).max() < 1e-10


@pytest.mark.parametrize("n", [1, 2, 5, 33, 100])
def test_syev_against_library(n):
    a, _, _ = W.spd(n, 1e3, 10 + n)
    lam, q = oracle.syev(a)
    ref = np.linalg.eigvalsh(a)
    assert np.abs(lam - ref).max() < 1e-13 * np.abs(ref).max() * n
    assert np.linalg.norm(q.T @ q - np.eye(n)) < 1e-13 * n
    assert np.linalg.norm((q * lam) @ q.T - a) < 1e-13 * n * np.linalg.norm(a)


def test_syev_single_precision_backward_error():
    a, _, _ = W.spd(80, 1e2, 5)
    lam, q = oracle.syev(a.astype(np.float32), single=True)
    assert lam.dtype == np.float32 and q.dtype == np.float32
    q64 = q.astype(np.float64)
    assert np.linalg.norm(q64.T @ q64 - np.eye(80)) < 80 * 6e-8 * 10
    assert np.linalg.norm((q64 * lam) @ q64.T - a) < 80 * 6e-8 * 10 * np.linalg.norm(a)


def test_against_scipy_sqrtm():
    import scipy.linalg as sl
    a = W.nonsym_shifted(60, 5)
    x = oracle.sqrtm(a)
    assert oracle.relerr(x, np.real(sl.sqrtm(a))) < 1e-12


def test_against_mpmath_50_digits():
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 50
    r = rng(11)
    n = 5
    a = r.standard_normal((n, n)) + 3 * np.eye(n)
    x = oracle.sqrtm(a)
    xm = mp.sqrtm(mp.matrix(a.tolist()))
    ref = np.array([[complex(xm[i, j]) for j in range(n)] for i in range(n)]).real
    assert oracle.relerr(x, ref) < 1e-14


# ---------------------------------------------------------------------------
# Invariants of the principal root


def test_invariants_real_nonsymmetric():
    a = W.nonsym_shifted(50, 3)
    x = oracle.sqrtm(a)
    assert x.dtype == np.float64  # real A -> real X
    assert oracle.relres(x, a) < 1e-13
    comm = np.linalg.norm(x @ a - a @ x) / (np.linalg.norm(x) * np.linalg.norm(a))
    assert comm < 1e-14
    assert np.all(np.linalg.eigvals(x).real > 0)


def test_equivariance_permutation_transpose_scaling():
    a = W.nonsym_shifted(30, 4)
    x = oracle.sqrtm(a)
    p = rng(2).permutation(30)
    pm = np.eye(30)[p]
    assert oracle.relerr(oracle.sqrtm(pm @ a @ pm.T), pm @ x @ pm.T) < 1e-13
    assert oracle.relerr(oracle.sqrtm(a.T), x.T) < 1e-13
    assert oracle.relerr(oracle.sqrtm(16.0 * a), 4.0 * x) < 1e-13


def test_spd_root_is_spd():
    a, _, _ = W.spd(40, 1e3, 9)
    x = oracle.sqrtm_spd(a)
    assert np.array_equal(x, x.T)
    assert np.linalg.eigvalsh(x).min() > 0


# ---------------------------------------------------------------------------
# Sylvester, Alg. 1 recursion and the adjoint


def _tri(r, m, shift=3.0):
    return np.triu(r.standard_normal((m, m)) + 1j * r.standard_normal((m, m))) + shift * np.eye(m)


@pytest.mark.parametrize("m,n", [(1, 1), (3, 7), (8, 2), (9, 9), (12, 5)])
def test_trsyl_against_kronecker(m, n):
    r = rng(m * 13 + n)
    s, st = _tri(r, m), _tri(r, n)
    c = r.standard_normal((m, n)) + 1j * r.standard_normal((m, n))
    ref = oracle.kron_sylvester(s, st, c)
    assert np.abs(oracle.trsyl(s, st, c) - ref).max() < 1e-13


@pytest.mark.parametrize("m,n,blks", [(12, 12, 2), (12, 3, 2), (3, 12, 2), (11, 7, 3), (10, 10, 32)])
def test_rtrsyl_all_branches_against_kronecker(m, n, blks):
    # (12,3): row-only split (2n <= m); (3,12): column-only split (2m <= n);
    # (12,12), (11,7): the 2x2 split; (10,10,32): base case.
    r = rng(m + 100 * n + blks)
    s, st = _tri(r, m), _tri(r, n)
    c = r.standard_normal((m, n)) + 1j * r.standard_normal((m, n))
    ref = oracle.kron_sylvester(s, st, c)
    assert np.abs(oracle.rtrsyl(s, st, c, blks=blks) - ref).max() < 1e-13


def test_four_block_equations_hold():
    # One level of the partition in Eq. (partition): the four sub-equations are
    # satisfied by the blocks of the solution.
    r = rng(21)
    m, n = 10, 8
    s, st = _tri(r, m), _tri(r, n)
    c = r.standard_normal((m, n)) + 1j * r.standard_normal((m, n))
    y = oracle.trsyl(s, st, c)
    m1, n1 = m // 2, n // 2
    S11, S12, S22 = s[:m1, :m1], s[:m1, m1:], s[m1:, m1:]
    T11, T12, T22 = st[:n1, :n1], st[:n1, n1:], st[n1:, n1:]
    Y11, Y12, Y21, Y22 = y[:m1, :n1], y[:m1, n1:], y[m1:, :n1], y[m1:, n1:]
    C11, C12, C21, C22 = c[:m1, :n1], c[:m1, n1:], c[m1:, :n1], c[m1:, n1:]
    tol = 1e-12
    assert np.abs(S11 @ Y11 + Y11 @ T11 - (C11 - S12 @ Y21)).max() < tol
    assert np.abs(S11 @ Y12 + Y12 @ T22 - (C12 - S12 @ Y22 - Y11 @ T12)).max() < tol
    assert np.abs(S22 @ Y21 + Y21 @ T11 - C21).max() < tol
    assert np.abs(S22 @ Y22 + Y22 @ T22 - (C22 - Y21 @ T12)).max() < tol


@pytest.mark.parametrize("n,cplx", [(1, False), (6, False), (9, True)])
def test_adjoint_against_kronecker(n, cplx):
    r = rng(30 + n)
    if cplx:
        a, _ = W.complex_square(n, 40 + n)
        g = r.standard_normal((n, n)) + 1j * r.standard_normal((n, n))
    else:
        a = W.nonsym_shifted(n, 50 + n)
        g = r.standard_normal((n, n))
    x = oracle.sqrtm(a)
    ga = oracle.adjoint(x, g)
    ref = oracle.kron_adjoint(x, g)
    assert np.abs(ga - ref).max() < 1e-12 * np.abs(ref).max()


def test_adjoint_spd_closed_form_against_schur_route_and_kronecker():
    n = 9
    a, q, lam = W.spd(n, 1e3, 80)
    g = rng(81).standard_normal((n, n))
    x = (q * np.sqrt(lam)) @ q.T
    ref = oracle.kron_adjoint(x, g).real
    assert np.abs(oracle.adjoint_spd(q, lam, g) - ref).max() < 1e-11 * np.abs(ref).max()
    assert np.abs(oracle.adjoint(oracle.sqrtm(a), g) - ref).max() < 1e-10 * np.abs(ref).max()


def test_adjoint_against_central_differences():
    # <Gbar, d sqrtm(A)[E]> = <G, E> with G = adjoint(X, Gbar).
    n = 7
    a = W.nonsym_shifted(n, 60)
    r = rng(61)
    gbar = r.standard_normal((n, n))
    e = r.standard_normal((n, n))
    e /= np.linalg.norm(e)
    h = 1e-5
    fd = np.sum(gbar * (oracle.sqrtm(a + h * e) - oracle.sqrtm(a - h * e))) / (2 * h)
    g = oracle.adjoint(oracle.sqrtm(a), gbar)
    assert abs(fd - np.sum(g * e)) < 1e-8 * max(1.0, abs(fd))


# ---------------------------------------------------------------------------
# Convergence theorem (Sec. 3.1) in exact-ish arithmetic


def test_convergence_theorem_inequality():
    # Iteration vec(X_{k+1}) = vec(X_k) + B_Z^{-1} vec(A - X_k^2) with a frozen,
    # perturbed Z satisfies ||E_{k+1}|| <= 2||B_Z^-1|| ||E_Z|| ||E_k||
    #                                      + ||B_Z^-1|| ||E_k||^2.
    n = 6
    a = W.nonsym_shifted(n, 70)
    x = oracle.sqrtm(a)
    r = rng(71)
    z = x + 1e-3 * r.standard_normal((n, n))
    bz = np.kron(np.eye(n), z) + np.kron(z.T, np.eye(n))
    binv = np.linalg.inv(bz)
    nb = np.linalg.norm(binv, 2)
    ez = np.linalg.norm(z - x)
    xk = x + 1e-2 * r.standard_normal((n, n))
    for _ in range(6):
        ek = np.linalg.norm(xk - x)
        upd = binv @ (a - xk @ xk).reshape(-1, order="F")
        xk = xk + upd.reshape((n, n), order="F")
        ek1 = np.linalg.norm(xk - x)
        assert ek1 <= 2 * nb * ez * ek + nb * ek ** 2 + 1e-14
    assert np.linalg.norm(xk - x) < 1e-12


# ---------------------------------------------------------------------------
# Mixed-precision emulator against the paper's observations (Sec. 5.1)


def _obs():
    with open(os.path.join(GOLDEN, "paper_observations.json")) as f:
        return json.load(f)


@pytest.mark.parametrize("kappa,seed", [(1e2, 2), (1e4, 3)])
def test_emulator_spd_steps(kappa, seed):
    obs = _obs()["steps_not_ill_conditioned"]
    a, q, lam = W.spd(256, kappa, seed)
    res = oracle.emulate_mixed(a, tol=1e-13)
    assert res["status"] == "ok"
    assert obs["min"] <= res["steps"] <= obs["max"]
    xt = (q * np.sqrt(lam)[None, :]) @ q.T
    assert oracle.relerr(res["X"], xt) < 1e-12


def test_emulator_general_steps():
    obs = _obs()["steps_not_ill_conditioned"]
    a = W.nonsym_shifted(128, 5)
    res = oracle.emulate_mixed(a, tol=1e-13)
    assert res["status"] == "ok"
    assert obs["min"] <= res["steps"] <= obs["max"]
    assert oracle.relerr(res["X"], oracle.sqrtm(a)) < 1e-12


def test_emulator_complex_steps():
    a, b = W.complex_square(64, 6)
    res = oracle.emulate_mixed(a, tol=1e-13)
    assert res["status"] == "ok" and 1 <= res["steps"] <= 3
    assert oracle.relerr(res["X"], b) < 1e-12


def _theorem_constants(q, s, x_true):
    """||B_Z^-1||_2 and ||E_Z||_F of the convergence theorem (Sec. 3.1) for the
    frozen Z = Q diag(s) Q^T, formed in float64 from the factor.  For a
    symmetric Z, B_Z = I kron Z + Z kron I has eigenvalues z_i + z_j, so
    ||B_Z^-1||_2 = 1 / (2 min_i z_i)."""
    q = np.asarray(q, dtype=np.float64)
    z = (q * np.asarray(s, dtype=np.float64)[None, :]) @ q.T
    z = 0.5 * (z + z.T)
    binv = 1.0 / (2.0 * np.linalg.eigvalsh(z).min())
    return binv, float(np.linalg.norm(z - x_true))


@pytest.mark.slow
def test_emulator_hilbert_rate_matches_convergence_theorem():
    """Table 1 set VII, Sec. 5.1: H_1024 + 1e-6 I converges, slowly.  The
    paper reports about 11-12 sweeps with its LAPACK single-precision
    eigensolver; the count depends on that solver's error E_Z through the
    theorem's rate 2 ||B_Z^-1|| ||E_Z||_F.  Pinned here: every observed error
    contraction obeys the theorem's bound for this emulator's own FP32 factor,
    and the sweep count lies between 'clearly more than the 1-3 of
    well-conditioned inputs' and the count the theorem's rate allows."""
    obs = _obs()
    h = obs["hilbert"]
    tol = obs["parameters"]["tol"]
    a = W.hilbert(h["n"], h["tau"])
    res = oracle.emulate_mixed(a, tol=tol, iterates=True)
    assert res["status"] == "ok"
    k = oracle.scale_exponent(a)
    asc = a / 4.0 ** k
    lam, q = oracle.syev(asc.astype(np.float32), single=True)
    x_true = oracle.sqrtm_spd(asc)
    binv, ez = _theorem_constants(q, np.sqrt(lam), x_true)
    rho_inf = 2 * binv * ez
    assert rho_inf < 1  # the theorem guarantees convergence
    errs = [np.linalg.norm(xk / 2.0 ** k - x_true) for xk in res["iterates"]]
    floor = 1e3 * np.finfo(float).eps * np.linalg.norm(x_true) * np.sqrt(binv)
    for e0, e1 in zip(errs[:-1], errs[1:]):
        if e1 > floor:
            assert e1 <= binv * (2 * ez + e0) * e0 * (1 + 1e-6)
    # sweeps that the theorem's asymptotic rate allows after the first
    # correction, starting from the first corrected residual
    allowed = 1 + int(np.ceil(np.log(res["hist"][1] / tol) / np.log(1.0 / rho_inf)))
    assert h["steps_approx"][1] <= allowed + 1   # the paper's count is within the bound
    assert 5 <= res["steps"] <= allowed


@pytest.mark.slow
def test_emulator_hilbert_threshold_no_principal_then_divergence():
    """Sec. 5.1: below a regularisation threshold the mixed method fails.  In
    FP32 the threshold shows up two ways: for tau <= 2.5e-7 (the paper's
    1e-7 included) the FP32 eigensolver returns an eigenvalue <= 0 of the
    positive definite H + tau I, so the float factor has no principal root
    (NO_PRINCIPAL at that precision); just above it, at tau = 2.8e-7, the
    factor is positive but the theorem's rate exceeds 1 and the residual grows
    on two consecutive sweeps (DIVERGED)."""
    tol = _obs()["parameters"]["tol"]
    n = _obs()["hilbert"]["n"]
    for tau in (_obs()["hilbert_divergence"]["tau_below"], 2e-7):
        a = W.hilbert(n, tau)
        assert np.linalg.eigvalsh(a).min() > 0
        assert oracle.emulate_mixed(a, tol=tol)["status"] == "no_principal"
    a = W.hilbert(n, 2.8e-7)
    res = oracle.emulate_mixed(a, tol=tol)
    assert res["status"] == "diverged"
    hst = res["hist"]
    assert hst[-1] > hst[-2] > hst[-3] and hst[-1] <= 10 * hst[0]
    k = oracle.scale_exponent(a)
    asc = a / 4.0 ** k
    lam, q = oracle.syev(asc.astype(np.float32), single=True)
    assert lam.min() > 0
    binv, ez = _theorem_constants(q, np.sqrt(lam), oracle.sqrtm_spd(asc))
    assert 2 * binv * ez > 1
    # the best iterate is returned
    assert oracle.relres(res["X"], a) == pytest.approx(min(hst), rel=1e-6)


def test_stop_rule_every_branch():
    """The divergence / stagnation reading of Sec. 5.1 ('diverges in our
    tests'), one history per branch, in the order the rule tests them."""
    rule = oracle._stop_rule
    assert rule([1e-3]) is None
    assert rule([1e-3, np.nan]) == "diverged"
    assert rule([1e-3, np.inf]) == "diverged"
    assert rule([1e-3, 2e-2]) == "diverged"                  # > 10x the first residual
    assert rule([1e-3, 2e-3]) is None                        # one growth is tolerated
    assert rule([1e-3, 2e-3, 3e-3]) == "diverged"            # two consecutive growths
    assert rule([1e-3, 9.5e-4, 9.1e-4]) == "not_converged"  # two ratios above 0.9
    assert rule([1e-3, 9.5e-4, 8e-4]) is None                # second ratio 0.84
    assert rule([1e-3, 1e-4, 9.5e-5]) is None                # one slow sweep only


def _spd_with_factor(n, seed, lam_range=(0.5, 2.0)):
    a, q, lam = W.spd_range(n, lam_range[0], lam_range[1], seed)
    return a, q, lam


# Scalar picture in the eigenbasis (exact Q): a component with eigenvalue
# lam and frozen root s evolves as e <- e (1 - (2 sqrt(lam) + e) / (2 s)), so
# s = sqrt(lam) / c gives the linear factor 1 - c.
FROZEN_ROOT_CASES = {
    # c: factor; start perturbation; expected status and the rule that fires
    "diverged_growth": (2.2, 1e-3, "diverged"),       # factor -1.2: grows twice
    "diverged_10x": (20.0, 1e-3, "diverged"),         # factor -19: > 10x the first residual
    "diverged_nonfinite": (None, 1e-3, "diverged"),   # s = 1e-300: the correction overflows
    "stagnated": (1.95, 1e-3, "not_converged"),       # factor -0.95: ratio above 0.9 twice
}


def frozen_root_case(name, n=64, seed=11):
    """SPD A = Q diag(lam) Q^T (k = 0), a factor with exact Q whose root s_0 is
    wrong by the case's factor, and a start X_0 = X + delta q_0 q_0^T."""
    c, delta, _ = FROZEN_ROOT_CASES[name]
    a, q, lam = _spd_with_factor(n, seed)
    s = np.sqrt(lam).copy()
    s[0] = 1e-300 if c is None else np.sqrt(lam[0]) / c
    x_true = (q * np.sqrt(lam)[None, :]) @ q.T
    x0 = x_true + delta * np.outer(q[:, 0], q[:, 0])
    return a, q, s, x0, x_true


@pytest.mark.parametrize("name", sorted(FROZEN_ROOT_CASES))
def test_emulator_frozen_root_statuses_and_theorem(name):
    """Failure statuses of the refinement with a deliberately wrong frozen
    root.  Each step obeys the first inequality of the convergence theorem
    (Sec. 3.1), ||E_{k+1}|| <= 2 ||B_Z^-1|| ||E_Z|| ||E_k|| + ||B_Z^-1|| ||E_k||^2,
    while it is finite, and the rule of the case fires."""
    a, q, s, x0, x_true = frozen_root_case(name)
    res = oracle.emulate_mixed(a, low="fp64", factor={"Q": q, "s": s}, x0=x0, tol=1e-13,
                               iterates=True)
    assert res["status"] == FROZEN_ROOT_CASES[name][2]
    hst = res["hist"]
    if name == "diverged_growth":
        assert hst[-1] > hst[-2] > hst[-3] and max(hst) <= 10 * hst[0]
    elif name == "diverged_10x":
        assert len(hst) == 2 and hst[1] > 10 * hst[0]
    elif name == "diverged_nonfinite":
        assert not np.isfinite(hst[-1]) and all(np.isfinite(hst[:-1]))
    else:
        assert len(hst) == 3 and hst[1] > 0.9 * hst[0] and hst[2] > 0.9 * hst[1]
    # best iterate returned
    best = int(np.argmin(hst))
    assert np.array_equal(res["X"], res["iterates"][best])
    if name != "diverged_nonfinite":
        binv, ez = _theorem_constants(q, s, x_true)
        errs = [np.linalg.norm(xk - x_true) for xk in res["iterates"]]
        for e0, e1 in zip(errs[:-1], errs[1:]):
            assert e1 <= (2 * binv * ez * e0 + binv * e0 ** 2) * (1 + 1e-9) + 1e-13


def test_emulator_failure_statuses():
    assert oracle.emulate_mixed(np.array([[np.nan, 0], [0, 1.0]]))["status"] == "nonfinite"
    res = oracle.emulate_mixed(W.spd(64, 1e4, 1)[0], maxit=0)
    assert res["status"] == "not_converged" and res["steps"] == 0


# ---------------------------------------------------------------------------
# The parallel oracle computes exactly what the serial one does


def test_parallel_oracle_bitwise_equals_serial():
    """OpenMP threads and the deferred application of the QR rotations change
    only which entries are updated when; each entry receives the same
    operations in the same order, so the results are bitwise equal to the
    plain serial order (immediate rotations, one thread).  Covered: a real
    and a complex Schur form, one that splits in the middle (the QR starts on
    a lower block and later works on the upper one), the triangular root, the
    symmetric eigendecomposition and the full square root."""
    r = rng(7)
    n = 150
    real = 2 * np.eye(n) + r.standard_normal((n, n)) / np.sqrt(n)
    split = real.copy()
    split[n // 2 + 1:, :n // 2 + 1] = 0
    cplx = r.standard_normal((n, n)) + 1j * r.standard_normal((n, n))
    spd, _, _ = W.spd(n + 7, 1e4, 2)

    def run():
        out = []
        for m in (real, split, cplx):
            t, q = oracle.schur(m)
            out += [t, q]
        out.append(oracle.trsqrt(out[0]))
        out += list(oracle.syev(spd))
        out.append(oracle.sqrtm(real))
        return out

    with oracle.execution(threads=1, deferred=False):
        ref = run()
    for threads in (2, 5):
        with oracle.execution(threads=threads, deferred=True):
            got = run()
        for u, v in zip(ref, got):
            assert np.array_equal(u, v)


def test_table1_families_structure_and_shift():
    """Table 1 generators: symmetric sets are exactly symmetric, the shift
    reading puts the whole spectrum in the open right half-plane, set VII is
    the Hilbert matrix plus 1e-6 I."""
    for sid in ("I", "II", "V", "VI"):
        a, shift = W.table1(sid, 5, n=160)
        sigma = np.sqrt(1 / 12.0) if sid in ("I", "V") else 1.0
        sym = sid in ("V", "VI")
        assert np.array_equal(a, a.T) == sym
        assert shift == pytest.approx((2.2 if sym else 1.1) * sigma * np.sqrt(160) + 1.0)
        assert np.linalg.eigvals(a).real.min() > 0
    h, tau = W.table1("VII", 0, n=12)
    assert tau == 1e-6 and h[2, 4] == pytest.approx(1.0 / 7.0) and h[0, 0] == 1.0 + 1e-6


# ---------------------------------------------------------------------------
# Matrix cube roots (Sec. 4, p = 3)


def _cube_root_pair(n, seed, cplx=True):
    """A = B^3 with B = Q (D + N) Q^H, D uniform in |z - 2| < 1 (so
    |arg| < 30 degrees and B is the principal cube root of A)."""
    r = rng(seed)
    z = r.standard_normal((n, n)) + (1j * r.standard_normal((n, n)) if cplx else 0)
    q, _ = np.linalg.qr(z)
    rad = np.sqrt(r.uniform(size=n))
    ang = 2 * np.pi * r.uniform(size=n)
    d = 2.0 + rad * np.exp(1j * ang)
    if not cplx:
        d = 2.0 + rad * np.cos(ang)
    nn = np.triu(r.standard_normal((n, n)), 1) * (0.1 / np.sqrt(n))
    b = q @ (np.diag(d) + nn) @ q.conj().T
    return b @ b @ b, b


def test_cube_root_diagonal_and_2x2_closed_forms():
    d = np.array([8.0, 0.125, 2.0 + 1j, -3.0 + 1e-3j, -3.0 - 1e-3j, 1j, 1e-9])
    x = oracle.rootm3(np.diag(d))
    expect = d.astype(np.complex128) ** (1.0 / 3.0)  # numpy's principal branch
    assert np.allclose(np.diag(x), expect, rtol=1e-14, atol=0)
    assert np.all(np.abs(np.angle(np.diag(x))) < np.pi / 3)
    # [[a, b], [0, c]]^(1/3) = [[a^1/3, b / (a^2/3 + a^1/3 c^1/3 + c^2/3)], [0, c^1/3]]
    a, b, c = 2.0 + 1j, -0.5 + 3j, 0.3 - 0.1j
    u = oracle.trroot3(np.array([[a, b], [0, c]]))
    ra, rc = a ** (1 / 3), c ** (1 / 3)
    assert np.abs(u - np.array([[ra, b / (ra * ra + ra * rc + rc * rc)], [0, rc]])).max() <= 1e-15 * 8


@pytest.mark.parametrize("cplx", [True, False])
def test_cube_root_known_root_library_and_invariants(cplx):
    import scipy.linalg as sl
    a, b = _cube_root_pair(60, 31 + cplx, cplx)
    if not cplx:
        a, b = a.real, b.real
    x = oracle.rootm3(a)
    assert np.iscomplexobj(x) == cplx
    assert oracle.relerr(x, b) <= 1e-12
    assert np.linalg.norm(x @ x @ x - a) / np.linalg.norm(a) <= 1e-13
    assert np.linalg.norm(x @ a - a @ x) / (np.linalg.norm(x) * np.linalg.norm(a)) <= 1e-14
    assert np.all(np.abs(np.angle(np.linalg.eigvals(x))) < np.pi / 3)
    xs = sl.fractional_matrix_power(a, 1.0 / 3.0)  # Schur-Pade, an independent method
    assert oracle.relerr(x, xs) <= 1e-11


@pytest.mark.parametrize("m,n,blks", [(9, 7, 64), (9, 7, 2), (40, 6, 4), (5, 37, 4), (33, 29, 8)])
def test_rtrsyl3_every_branch_against_kronecker(m, n, blks):
    r = rng(100 + m + n)
    s = np.triu(r.standard_normal((m, m)) + 1j * r.standard_normal((m, m))) * 0.3 + 2 * np.eye(m)
    st = np.triu(r.standard_normal((n, n)) + 1j * r.standard_normal((n, n))) * 0.3 + 2 * np.eye(n)
    c = r.standard_normal((m, n)) + 1j * r.standard_normal((m, n))
    ref = oracle.kron_sylvester3(s, st, c)
    for y in (oracle.trsyl3(s, st, c), oracle.rtrsyl3(s, st, c, blks=blks)):
        assert oracle.relerr(y, ref) <= 1e-13


def test_rtrsyl3_block_equations_of_one_level():
    """The four block equations of Sec. 4 hold for the blocks of the
    recursion's solution (one level, split at floor(m/2), floor(n/2))."""
    r = rng(7)
    m = n = 24
    s = np.triu(r.standard_normal((m, m)) + 1j * r.standard_normal((m, m))) * 0.3 + 2 * np.eye(m)
    st = np.triu(r.standard_normal((n, n)) + 1j * r.standard_normal((n, n))) * 0.3 + 2 * np.eye(n)
    c = r.standard_normal((m, n)) + 1j * r.standard_normal((m, n))
    y = oracle.rtrsyl3(s, st, c, blks=4)
    h, g = m // 2, n // 2
    S11, S12, S22 = s[:h, :h], s[:h, h:], s[h:, h:]
    T11, T12, T22 = st[:g, :g], st[:g, g:], st[g:, g:]
    Y11, Y12, Y21, Y22 = y[:h, :g], y[:h, g:], y[h:, :g], y[h:, g:]
    C11, C12, C21, C22 = c[:h, :g], c[:h, g:], c[h:, :g], c[h:, g:]

    def op(sa, yy, tb):
        return sa @ sa @ yy + sa @ yy @ tb + yy @ tb @ tb

    s2_12 = S11 @ S12 + S12 @ S22
    t2_12 = T11 @ T12 + T12 @ T22
    tol = 1e-12 * np.linalg.norm(c)
    assert np.linalg.norm(op(S22, Y21, T11) - C21) <= tol
    assert np.linalg.norm(op(S11, Y11, T11) - (C11 - s2_12 @ Y21 - S12 @ Y21 @ T11)) <= tol
    assert np.linalg.norm(op(S22, Y22, T22) - (C22 - Y21 @ t2_12 - S22 @ Y21 @ T12)) <= tol
    rhs12 = (C12 - s2_12 @ Y22 - S12 @ Y22 @ T22 - Y11 @ t2_12 - (S11 @ Y11 + S12 @ Y21) @ T12)
    assert np.linalg.norm(op(S11, Y12, T22) - rhs12) <= tol


def test_emulator_cube_root_converges_to_the_known_root():
    a, b = _cube_root_pair(80, 41)
    res = oracle.emulate_mixed_root3(a, tol=1e-13)
    assert res["status"] == "ok" and 1 <= res["steps"] <= 3
    assert oracle.relerr(res["X"], b) <= 1e-12
    assert oracle.relerr(res["X"], oracle.rootm3(a)) <= 1e-12
