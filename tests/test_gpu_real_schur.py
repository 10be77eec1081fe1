"""Real input on the general path through the real Schur form (remark on
real input in Sec. 2.2.1): real double-shift QR, quasi-triangular root with
2x2 blocks and the quasi-triangular Sylvester solves on tiles that never cut
a 2x2 block.  Compared with the oracle's float64 real-Schur root, the
oracle's complex route, the library's complex route, and the emulator's
correction counts."""

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu


def _c2(n, seed):
    rng = np.random.default_rng(seed)
    return 2.0 * np.eye(n) + rng.standard_normal((n, n)) / np.sqrt(n)


@pytest.mark.parametrize("n", [1, 2, 5, 33, 97, 257])
def test_real_route_root_matches_oracle(n):
    import torch
    import paper_2607_12430_amd as msq
    a = _c2(n, 100 + n)
    print(f"[real-schur] n={n}", flush=True)
    x, info = msq.sqrtm(torch.from_numpy(a).cuda(), structure="general")
    assert info["status"] == "ok", info
    xh = x.cpu().numpy()
    assert O.relres(xh, a) <= 1e-13
    assert O.relerr(xh, O.sqrtm_real(a)) <= 1e-12


@pytest.mark.parametrize("prec", ["fp32", "fp64", "bf16split"])
def test_real_route_factor_is_a_real_schur_form(prec):
    import torch
    import paper_2607_12430_amd as msq
    n = 211
    a = _c2(n, 7)
    f = msq.factor(torch.from_numpy(a).cuda(), prec=prec, structure="general")
    q, u, k = f.export(single=prec != "fp64", structure="general")
    q, u = q[0].astype(np.float64), u[0].reshape(n, n).T.astype(np.float64)
    tol = 1e-12 if prec == "fp64" else 5e-5
    assert np.linalg.norm(q.T @ q - np.eye(n)) <= tol * n
    # U is quasi-upper-triangular with standardised 2x2 blocks
    assert np.all(np.tril(u, -2) == 0)
    sub = np.nonzero(np.diag(u, -1))[0]
    assert len(sub) >= 4 and np.all(np.diff(sub) >= 2)
    for i in sub:
        assert u[i, i] > 0 and u[i, i + 1] * u[i + 1, i] < 0
    # Q U^2 Q^T reproduces the input / 4^k to the factor's precision (the
    # library reads the row-major host array column-major, i.e. factors A^T)
    rec = q @ u @ u @ q.T * 4.0 ** k
    assert np.linalg.norm(rec - a.T) <= (1e-12 if prec == "fp64" else 2e-5) * np.linalg.norm(a)


@pytest.mark.parametrize("n", [300, 1000])
def test_real_route_agrees_with_complex_route_and_emulator(n):
    import torch
    import paper_2607_12430_amd as msq
    a = _c2(n, 3 * n)
    ad = torch.from_numpy(a).cuda()
    print(f"[real-schur] routes n={n}", flush=True)
    xr, ir = msq.sqrtm(ad, structure="general", fallback=False)
    xc, ic = msq.sqrtm(ad, structure="general", fallback=False, real_schur=False)
    assert ir["status"] == "ok" and ic["status"] == "ok"
    assert O.relerr(xr.cpu().numpy(), xc.cpu().numpy()) <= 1e-12
    emu = O.emulate_mixed(a, structure="general", schur_form="real")
    assert emu["status"] == "ok"
    assert abs(ir["steps"] - emu["steps"]) <= 1, (ir["relres_hist"], emu["hist"])
    # the first residual is that of a float factor
    assert 1e-9 < ir["relres_hist"][0] < 1e-4


def test_real_route_negative_eigenvalue_has_no_principal_root():
    import torch
    import paper_2607_12430_amd as msq
    n = 64
    rng = np.random.default_rng(5)
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    t = np.triu(rng.standard_normal((n, n)) * 0.1, 1) + np.diag(rng.uniform(1.0, 2.0, n))
    t[10, 10] = -1.5
    a = q @ t @ q.T
    _, info = msq.sqrtm(torch.from_numpy(a).cuda(), structure="general", allow_fail=True)
    assert info["status"] == "no_principal", info


def test_real_route_backward_matches_oracle_adjoint():
    import torch
    import paper_2607_12430_amd as msq
    n = 96
    a = _c2(n, 17)
    rng = np.random.default_rng(18)
    gbar = rng.standard_normal((n, n))
    ad = torch.from_numpy(a).cuda()
    x, info, f = msq.sqrtm(ad, structure="general", keep_factor=True)
    assert info["status"] == "ok"
    g, binfo = msq.sqrtm_backward(f, x, torch.from_numpy(gbar).cuda())  # raises on failure
    assert binfo["relres"] <= 1e-13 and binfo["steps"] >= 1, binfo
    ref = O.adjoint(x.cpu().numpy(), gbar)
    assert np.linalg.norm(g.cpu().numpy() - ref) <= 1e-10 * np.linalg.norm(ref)


def _blocks_at(n, starts, seed):
    """Real matrix Q U^2 Q^T whose real Schur form has 2x2 blocks starting at
    the given indices (U quasi-triangular with complex pairs there), so that
    blocks can be placed across the solvers' 32-row tile boundaries."""
    rng = np.random.default_rng(seed)
    u = np.triu(rng.standard_normal((n, n)) * 0.2, 1)
    i = 0
    while i < n:
        if i in starts and i + 1 < n:
            a = rng.uniform(0.6, 1.6)
            b = rng.uniform(0.4, 1.2)
            u[i, i] = u[i + 1, i + 1] = a
            u[i, i + 1] = b
            u[i + 1, i] = -rng.uniform(0.4, 1.2)
            i += 2
        else:
            u[i, i] = rng.uniform(0.6, 1.6)
            i += 1
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return q @ (u @ u) @ q.T, q @ u @ q.T


@pytest.mark.parametrize("n", [3, 4, 31, 32, 33, 63, 64, 65, 130])
def test_real_route_small_and_boundary_sizes(n):
    """Orders around the 32-row tiles and the smallest orders (one 2x2 block,
    a 2x2 block plus a 1x1, two blocks) against the known root."""
    import torch
    import paper_2607_12430_amd as msq
    starts = {0, 30, 31, 62, 63, 95, 126} if n > 4 else {0}
    a, root = _blocks_at(n, starts, 400 + n)
    print(f"[real-schur] boundary n={n}", flush=True)
    for prec in ("fp32", "fp64"):
        x, info = msq.sqrtm(torch.from_numpy(a.T.copy()).cuda(), structure="general", prec=prec,
                            fallback=False)
        assert info["status"] == "ok", (prec, info)
        xh = x.cpu().numpy().T
        assert O.relres(xh, a) <= 1e-13
        assert O.relerr(xh, root) <= 1e-11


def test_real_route_factor_then_refine_from_caller_iterate():
    """msqrt_factor + msqrt_refine on the real route: from X_0 of the factor,
    and from the root of a nearby matrix (the caller's iterate)."""
    import torch
    import paper_2607_12430_amd as msq
    n = 300
    a = _c2(n, 901)
    at = torch.from_numpy(a.T.copy()).cuda()
    f = msq.factor(at, prec="fp32", structure="general")
    x = torch.empty_like(at)
    info = msq.refine(f, at, x, init_from_factor=True)
    assert info["status"] == "ok" and 1 <= info["steps"] <= 3
    xr = O.sqrtm_real(a)
    assert O.relerr(x.cpu().numpy().T, xr) <= 1e-12
    # caller iterate: the root of A + 1e-6 E, refined against A with A's factor
    rng = np.random.default_rng(902)
    b = a + 1e-6 * rng.standard_normal((n, n)) / np.sqrt(n)
    xb = torch.from_numpy(O.sqrtm_real(b).T.copy()).cuda()
    info2 = msq.refine(f, at, xb, init_from_factor=False)
    assert info2["status"] == "ok" and info2["steps"] >= 1
    assert O.relerr(xb.cpu().numpy().T, xr) <= 1e-12
