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
