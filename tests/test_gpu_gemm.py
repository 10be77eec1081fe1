"""The MFMA GEMMs element by element against a float64 product: the float
kernels for ragged sizes and every transpose (|C - AB| <= 4 k 2^-24 |A||B|),
including single full products large enough for the 256 x 256-tile kernel
(K >= 2048, more than two 128-tiles per CU, one 256-tile on 90-100% of the
CUs),
and the symmetric-output (mirroring) launches in float and double at orders
whose triangle of 128-tiles exceeds two workgroups per CU, where the 192 x
192-tile kernels run (float: 4 k 2^-24 |A||A|^T; double: 4 k 2^-53)."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("ta,tb", [(False, False), (True, False), (False, True), (True, True)])
@pytest.mark.parametrize("m,n,k", [(1601, 1543, 301), (1537, 2113, 257), (2048, 2048, 512),
                                   (3900, 4000, 2100), (4096, 4096, 2056)])
def test_wide_tile_float_gemm(ta, tb, m, n, k):
    import paper_2607_12430_amd as msq
    rng = np.random.Generator(np.random.PCG64(m + 3 * n + 7 * k + 11 * ta + 13 * tb))
    a = rng.standard_normal((k, m) if ta else (m, k)).astype(np.float32)
    b = rng.standard_normal((n, k) if tb else (k, n)).astype(np.float32)
    a64 = a.astype(np.float64).T if ta else a.astype(np.float64)
    b64 = b.astype(np.float64).T if tb else b.astype(np.float64)
    ref = a64 @ b64
    scale = np.abs(a64) @ np.abs(b64)
    c = msq.test_gemm_f32(a, b, split=False, ta=ta, tb=tb).astype(np.float64)
    assert np.max(np.abs(c - ref) / scale) <= 4.0 * k * 2.0 ** -24


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("n,k", [(4000, 300), (4096, 257), (1700, 64)])
def test_symmetric_output_gemm(prec, n, k):
    import paper_2607_12430_amd as msq
    rng = np.random.Generator(np.random.PCG64(n + 5 * k + (prec == "fp64")))
    a = rng.standard_normal((n, k))
    if prec == "fp32":
        a = a.astype(np.float32)
    a64 = a.astype(np.float64)
    ref = a64 @ a64.T
    scale = np.abs(a64) @ np.abs(a64).T
    c = msq.test_syrk(a, prec=prec).astype(np.float64)
    u = 2.0 ** -24 if prec == "fp32" else 2.0 ** -53
    assert np.max(np.abs(c - ref) / scale) <= 4.0 * k * u
    assert np.array_equal(c, c.T)  # every element mirrored exactly
