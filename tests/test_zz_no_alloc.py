"""msqrt_refine_noalloc (static device scratch, no allocation) against
msqrt_refine through the C-ABI: same status, corrections, residual history
and iterate, on consecutive calls that reuse the scratch, the later ones
smaller."""

import numpy as np
import pytest

import oracle
import workloads as W
from test_oracle_pins import frozen_root_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def msq():
    import paper_2607_12430_amd as m
    return m


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _both(msq, f, a, x0, **kw):
    xa, xb = _dev(x0), _dev(x0)
    ia = msq.refine(f, _dev(a), xa, allow_fail=True, **kw)
    ib = msq.refine_noalloc(f, _dev(a), xb, allow_fail=True, **kw)
    return ia, ib, xa.cpu().numpy(), xb.cpu().numpy()


def _same(ia, ib, xa, xb):
    assert ib["status"] == ia["status"]
    assert ib["steps"] == ia["steps"]
    assert ib["relres_hist"] == ia["relres_hist"]
    assert np.array_equal(xa, xb)


def test_noalloc_matches_refine_on_consecutive_calls(msq):
    # larger call first, then smaller ones reusing the same scratch
    for n, kappa, seed in ((300, 1e4, 31), (130, 1e2, 32), (37, 1e4, 33)):
        a, q, lam = W.spd(n, kappa, seed)
        lam32, q32 = oracle.syev(a.astype(np.float32), single=True)
        f = msq.factor_wrap(q32, np.sqrt(lam32).astype(np.float32), prec="fp32")
        ia, ib, xa, xb = _both(msq, f, a, np.zeros((n, n)), init_from_factor=True)
        _same(ia, ib, xa, xb)
        assert ib["status"] == "ok" and oracle.relres(xb, a) <= 1e-13
        assert oracle.relerr(xb, (q * np.sqrt(lam)) @ q.T) <= 1e-11


def test_noalloc_float64_factor_and_divergence(msq):
    # float64 factor, caller start, and a diverging frozen root (the best
    # iterate is restored from the scratch)
    a, q, s, x0, _ = frozen_root_case("diverged_growth")
    x0 = 0.5 * (x0 + x0.T)
    f = msq.factor_wrap(q, s, prec="fp64")
    ia, ib, xa, xb = _both(msq, f, a, x0, init_from_factor=False)
    _same(ia, ib, xa, xb)
    assert ib["status"] == "diverged"
    n = 24
    a, q, lam = W.spd(n, 1e4, 34)
    lam64, q64 = oracle.syev(a)
    f = msq.factor_wrap(q64, np.sqrt(lam64), prec="fp64")
    ia, ib, xa, xb = _both(msq, f, a, np.zeros((n, n)), init_from_factor=True)
    _same(ia, ib, xa, xb)
    assert ib["status"] == "ok"


def test_noalloc_rejects_oversize_and_general_factors(msq):
    import torch
    n = 1800  # float64 factor: 24 n^2 bytes > 64 MiB
    q = np.eye(n)
    f = msq.factor_wrap(q, np.ones(n), prec="fp64")
    a = _dev(np.eye(n))
    x = torch.full((n, n), 3.0, dtype=torch.float64, device="cuda")
    info = msq.refine_noalloc(f, a, x, allow_fail=True)
    assert info["status"] == "invalid_arg"
    assert bool((x == 3.0).all())
    g = W.nonsym_shifted(40, 35)
    _, _, fg = msq.sqrtm(_dev(g), keep_factor=True)
    x = torch.zeros((40, 40), dtype=torch.float64, device="cuda")
    info = msq.refine_noalloc(fg, _dev(g), x, allow_fail=True)
    assert info["status"] == "unsupported"
