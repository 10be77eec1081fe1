"""CPU oracle for the mixed-precision matrix square root.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the library itself.  It shares no code
with the HIP path.

What it computes (each function cites the passage of the paper it follows):

* ``sqrtm``: the principal square root (Sec. 1 definition) by the Schur method
  in float64/complex128: complex Schur form, column recurrence Eq. (subst),
  X = Q S Q^H (Sec. 2.1).  Real input returns the real part after asserting
  that the imaginary part is at rounding level.
* ``sqrtm_spd``: the SPD route of Alg. 3 in float64: spectral decomposition,
  s_i = lam_i^{1/2}, X = Q S Q^T.
* ``trsyl`` / ``rtrsyl``: the triangular Sylvester equation S Y + Y St = C
  (Eq. (triangsylv)) by back-substitution, and Alg. 1's block recursion.
* ``adjoint``: G with X^H G + G X^H = Gbar, the adjoint of the Frechet
  derivative of the square root (the correction operator B_X of Sec. 3.1).
* ``kron_sylvester``: brute-force Kronecker solve of S Y + Y St = C
  (vec form of Sec. 3.1) for tiny sizes.
* ``emulate_mixed``: Alg. 2 / Alg. 3 with the factorisation run by this
  module's own textbook routines in single precision and the residual and
  update in double precision, with the stopping rule of Alg. 2 and the
  divergence / stagnation rules stated below.  Used for step counts and the
  failure paths without a GPU.
* ``rootm3``, ``trroot3``, ``trsyl3`` / ``rtrsyl3``, ``emulate_mixed_root3``:
  the matrix cube root of Sec. 4 (Schur method, the generalized triangular
  Sylvester equation S^2 Y + S Y St + Y St^2 = C by substitution and by the
  block recursion, and the mixed-precision framework for p = 3).
* ``real_schur``, ``trsqrt_quasi``, ``trsyl_quasi`` / ``rtrsyl_quasi``,
  ``sqrtm_real``: the real route of the remark in Sec. 2.2.1 (real Schur form,
  quasi-triangular root and Sylvester solves, no 2x2 block cut by a split).
* ``mlp_*``: float64 forward/backward of the small precision-selector network.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

OK, NOCONV, NO_PRINCIPAL = 0, 1, 2


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        _lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        fp = ctypes.POINTER(ctypes.c_float)
        i = ctypes.c_int
        _lib.orc_schur_z.argtypes = [i, dp, dp]
        _lib.orc_schur_c.argtypes = [i, fp, fp]
        _lib.orc_trsqrt_z.argtypes = [i, dp, dp]
        _lib.orc_trsqrt_c.argtypes = [i, fp, fp]
        _lib.orc_sqrtm_z.argtypes = [i, dp, dp, dp, dp, dp]
        _lib.orc_syev_d.argtypes = [i, dp, dp, dp]
        _lib.orc_syev_s.argtypes = [i, fp, fp, fp]
        _lib.orc_trsyl_z.argtypes = [i, i, dp, dp, dp, dp]
        _lib.orc_trsyl_c.argtypes = [i, i, fp, fp, fp, fp]
        _lib.orc_rtrsyl_z.argtypes = [i, i, dp, dp, dp, i]
        _lib.orc_rtrsyl_c.argtypes = [i, i, fp, fp, fp, i]
        _lib.orc_adjoint_z.argtypes = [i, dp, dp, dp]
        _lib.orc_trroot3_z.argtypes = [i, dp, dp]
        _lib.orc_trroot3_c.argtypes = [i, fp, fp]
        _lib.orc_trsyl3_z.argtypes = [i, i, dp, dp, dp, dp]
        _lib.orc_rtrsyl3_z.argtypes = [i, i, dp, dp, dp, i]
        _lib.orc_rtrsyl3_c.argtypes = [i, i, fp, fp, fp, i]
        _lib.orc_rootm3_z.argtypes = [i, dp, dp, dp, dp, dp]
        for f in ("orc_trroot3_z", "orc_trroot3_c", "orc_rootm3_z"):
            getattr(_lib, f).restype = ctypes.c_int
        for f in ("orc_trsyl3_z", "orc_rtrsyl3_z", "orc_rtrsyl3_c"):
            getattr(_lib, f).restype = None
        _lib.orc_trsqrt_quasi_d.argtypes = [i, dp, dp]
        _lib.orc_trsqrt_quasi_s.argtypes = [i, fp, fp]
        _lib.orc_trsyl_quasi_d.argtypes = [i, i, dp, dp, dp, dp]
        _lib.orc_rtrsyl_quasi_d.argtypes = [i, i, dp, dp, dp, i]
        _lib.orc_rtrsyl_quasi_s.argtypes = [i, i, fp, fp, fp, i]
        _lib.orc_sqrt_2x2_d.argtypes = [dp, dp]
        for f in ("orc_trsqrt_quasi_d", "orc_trsqrt_quasi_s", "orc_sqrt_2x2_d"):
            getattr(_lib, f).restype = ctypes.c_int
        for f in ("orc_trsyl_quasi_d", "orc_rtrsyl_quasi_d", "orc_rtrsyl_quasi_s"):
            getattr(_lib, f).restype = None
        _lib.orc_set_threads.argtypes = [i]
        _lib.orc_set_threads.restype = None
        _lib.orc_get_threads.argtypes = []
        _lib.orc_get_threads.restype = i
        _lib.orc_set_deferred.argtypes = [i]
        _lib.orc_set_deferred.restype = None
        for f in ("orc_schur_z", "orc_schur_c", "orc_trsqrt_z", "orc_trsqrt_c", "orc_sqrtm_z",
                  "orc_syev_d", "orc_syev_s", "orc_adjoint_z"):
            getattr(_lib, f).restype = ctypes.c_int
        for f in ("orc_trsyl_z", "orc_trsyl_c", "orc_rtrsyl_z", "orc_rtrsyl_c"):
            getattr(_lib, f).restype = None
    return _lib


class OracleError(RuntimeError):
    pass


class execution:
    """Context manager selecting how the C++ routines run: `threads` OpenMP
    threads (None keeps the current count) and `deferred` (True: the QR
    rotations outside the active block and on Q are logged and applied later
    in parallel; False: applied at once, the plain serial order).  Every
    setting computes the same floating-point operations per entry, so the
    results are bitwise identical (pinned by a test)."""

    def __init__(self, threads=None, deferred=True):
        self.threads = threads
        self.deferred = deferred

    def __enter__(self):
        self._old = lib().orc_get_threads()
        if self.threads:
            lib().orc_set_threads(int(self.threads))
        lib().orc_set_deferred(1 if self.deferred else 0)
        return self

    def __exit__(self, *exc):
        lib().orc_set_threads(self._old)
        lib().orc_set_deferred(1)
        return False


def _f(a, dtype):
    return np.asfortranarray(np.asarray(a, dtype=dtype))


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _check(st, what):
    if st == NOCONV:
        raise OracleError(f"{what}: QR iteration did not converge")
    if st == NO_PRINCIPAL:
        raise OracleError(f"{what}: eigenvalue on the closed negative real axis; no principal root")


# ---------------------------------------------------------------------------
# Factorisations and the triangular square root


def schur(a, single=False):
    """Complex Schur form A = Q T Q^H.  Returns (T, Q)."""
    dt = np.complex64 if single else np.complex128
    ct = ctypes.c_float if single else ctypes.c_double
    t = _f(a, dt).copy(order="F")
    n = t.shape[0]
    q = np.zeros((n, n), dtype=dt, order="F")
    fn = lib().orc_schur_c if single else lib().orc_schur_z
    _check(fn(n, _ptr(t, ct), _ptr(q, ct)), "schur")
    return t, q


def trsqrt(t, single=False):
    """Square root of an upper triangular matrix by Eq. (subst)."""
    dt = np.complex64 if single else np.complex128
    ct = ctypes.c_float if single else ctypes.c_double
    t = _f(t, dt)
    n = t.shape[0]
    s = np.zeros((n, n), dtype=dt, order="F")
    fn = lib().orc_trsqrt_c if single else lib().orc_trsqrt_z
    _check(fn(n, _ptr(t, ct), _ptr(s, ct)), "trsqrt")
    return s


def syev(a, single=False):
    """Symmetric eigendecomposition A = Q diag(lam) Q^T, lam ascending."""
    dt = np.float32 if single else np.float64
    ct = ctypes.c_float if single else ctypes.c_double
    a = _f(a, dt)
    n = a.shape[0]
    lam = np.zeros(n, dtype=dt)
    q = np.zeros((n, n), dtype=dt, order="F")
    fn = lib().orc_syev_s if single else lib().orc_syev_d
    _check(fn(n, _ptr(a, ct), _ptr(lam, ct), _ptr(q, ct)), "syev")
    return lam, q


def sqrtm(a, return_factors=False, imag_tol=1e-12):
    """Principal square root by the float64 Schur method (Sec. 1, Sec. 2.1)."""
    a = np.asarray(a)
    is_real = not np.iscomplexobj(a)
    az = _f(a, np.complex128)
    n = az.shape[0]
    if n == 0:
        x = np.zeros((0, 0), dtype=a.dtype)
        return (x, None) if return_factors else x
    if not np.all(np.isfinite(az)):
        raise OracleError("sqrtm: non-finite input")
    x = np.zeros((n, n), dtype=np.complex128, order="F")
    q = np.zeros_like(x)
    t = np.zeros_like(x)
    s = np.zeros_like(x)
    dp = ctypes.c_double
    st = lib().orc_sqrtm_z(n, _ptr(az, dp), _ptr(x, dp), _ptr(q, dp), _ptr(t, dp), _ptr(s, dp))
    _check(st, "sqrtm")
    if is_real:
        nx = np.linalg.norm(x)
        ni = np.linalg.norm(x.imag)
        if nx > 0 and ni > imag_tol * nx:
            raise OracleError(f"sqrtm: real input gave imaginary part {ni / nx:.2e}")
        x = np.asfortranarray(x.real)
    if return_factors:
        return x, {"Q": q, "T": t, "S": s}
    return x


def sqrtm_spd(a):
    """SPD route of Alg. 3 in float64: A = Q diag(lam) Q^T, X = Q diag(lam^1/2) Q^T."""
    lam, q = syev(a)
    if np.any(lam <= 0):
        raise OracleError("sqrtm_spd: matrix is not positive definite")
    x = (q * np.sqrt(lam)[None, :]) @ q.T
    return np.asfortranarray(0.5 * (x + x.T))


# ---------------------------------------------------------------------------
# Matrix cube roots (Sec. 4, p = 3)


def trroot3(t, single=False):
    """U = T^{1/3} for upper triangular T: principal cube roots on the
    diagonal and the Schur-method recurrence for p = 3 (see oracle.cpp)."""
    dt = np.complex64 if single else np.complex128
    ct = ctypes.c_float if single else ctypes.c_double
    t = _f(t, dt)
    n = t.shape[0]
    u = np.zeros((n, n), dtype=dt, order="F")
    fn = lib().orc_trroot3_c if single else lib().orc_trroot3_z
    _check(fn(n, _ptr(t, ct), _ptr(u, ct)), "trroot3")
    return u


def rootm3(a, return_factors=False, imag_tol=1e-12):
    """Principal cube root (Sec. 4 definition: X^3 = A, eigenvalues in
    |arg z| < pi/3) by the float64 Schur method: A = Q T Q^H, U = T^{1/3},
    X = Q U Q^H.  Real input returns the real part after asserting that the
    imaginary part is at rounding level."""
    a = np.asarray(a)
    is_real = not np.iscomplexobj(a)
    az = _f(a, np.complex128)
    n = az.shape[0]
    if not np.all(np.isfinite(az)):
        raise OracleError("rootm3: non-finite input")
    x = np.zeros((n, n), dtype=np.complex128, order="F")
    q, t, u = np.zeros_like(x), np.zeros_like(x), np.zeros_like(x)
    dp = ctypes.c_double
    _check(lib().orc_rootm3_z(n, _ptr(az, dp), _ptr(x, dp), _ptr(q, dp), _ptr(t, dp), _ptr(u, dp)),
           "rootm3")
    if is_real:
        nx, ni = np.linalg.norm(x), np.linalg.norm(x.imag)
        if nx > 0 and ni > imag_tol * nx:
            raise OracleError(f"rootm3: real input gave imaginary part {ni / nx:.2e}")
        x = np.asfortranarray(x.real)
    return (x, {"Q": q, "T": t, "U": u}) if return_factors else x


def trsyl3(s, st, c):
    """S^2 Y + S Y St + Y St^2 = C (S, St upper triangular), unblocked
    substitution (complex128)."""
    s, st, c = _f(s, np.complex128), _f(st, np.complex128), _f(c, np.complex128)
    m, n = c.shape
    y = np.zeros((m, n), dtype=np.complex128, order="F")
    dp = ctypes.c_double
    lib().orc_trsyl3_z(m, n, _ptr(s, dp), _ptr(st, dp), _ptr(c, dp), _ptr(y, dp))
    return y


def rtrsyl3(s, st, c, blks=32, single=False):
    """The p = 3 block recursion of Sec. 4 for S^2 Y + S Y St + Y St^2 = C."""
    dt = np.complex64 if single else np.complex128
    ct = ctypes.c_float if single else ctypes.c_double
    s, st = _f(s, dt), _f(st, dt)
    y = _f(c, dt).copy(order="F")
    m, n = y.shape
    fn = lib().orc_rtrsyl3_c if single else lib().orc_rtrsyl3_z
    fn(m, n, _ptr(s, ct), _ptr(st, ct), _ptr(y, ct), int(blks))
    return y


def kron_sylvester3(s, st, c):
    """Brute force: (I kron S^2 + St^T kron S + (St^2)^T kron I) vec(Y) = vec(C),
    the vec form of the p = 3 correction operator (Sec. 4 with Sec. 3.1)."""
    s = np.asarray(s, dtype=np.complex128)
    st = np.asarray(st, dtype=np.complex128)
    c = np.asarray(c, dtype=np.complex128)
    m, n = c.shape
    big = (np.kron(np.eye(n), s @ s) + np.kron(st.T, s) + np.kron((st @ st).T, np.eye(m)))
    y = np.linalg.solve(big, c.reshape(-1, order="F"))
    return y.reshape((m, n), order="F")


def scale_exponent3(a):
    """k with A/8^k of Frobenius norm near sqrt(n): exact scaling for the
    cube root (X is scaled by 2^-k)."""
    n = a.shape[0]
    nrm = np.linalg.norm(a)
    if nrm == 0 or n == 0:
        return 0
    return int(np.round(np.log(nrm / np.sqrt(n)) / np.log(8.0)))


def emulate_mixed_root3(a, maxit=30, tol=1e-13, blks=32, iterates=False):
    """The Sec. 4 framework for p = 3: X_0 from the single-precision Schur
    cube root, residual R = A - X^3 in double precision, correction from
    S^2 Y + S Y S + Y S^2 = Q^H fl_l(R) Q in single precision (the p = 3
    block recursion), X += Q Y Q^H in double precision; stopping and
    divergence rules as in emulate_mixed (tol < 0 nullifies the stop)."""
    a = np.asarray(a)
    is_real = not np.iscomplexobj(a)
    if not np.all(np.isfinite(a)):
        return {"X": None, "steps": 0, "hist": [], "status": ST_NONFINITE}
    k = scale_exponent3(a)
    asc = a / (8.0 ** k)
    na = np.linalg.norm(asc)
    t, q = schur(asc.astype(np.complex64), single=True)
    d = np.diag(t)
    if np.any((d.imag == 0) & (d.real <= 0)):
        return {"X": None, "steps": 0, "hist": [], "status": ST_NO_PRINCIPAL}
    u = trroot3(t, single=True)
    qh = q.conj().T
    x0 = (q @ u @ qh).astype(np.complex128)
    x = x0.real.copy() if is_real else x0

    def correction(r):
        rl = r.astype(np.complex64)
        y = rtrsyl3(u, u, qh @ rl @ q, blks=blks, single=True)
        dx = (q @ y @ qh).astype(np.complex128)
        return dx.real if is_real else dx

    hist, seq = [], []
    best = (np.inf, x)
    status = ST_NOT_CONVERGED
    steps = 0
    with np.errstate(over="ignore", invalid="ignore"):
        for it in range(maxit + 1):
            if iterates:
                seq.append(x * (2.0 ** k))
            r = asc - x @ x @ x
            rr = float(np.linalg.norm(r) / na)
            hist.append(rr)
            if rr < best[0]:
                best = (rr, x)
            if tol < 0:
                if not np.isfinite(rr):
                    status = ST_DIVERGED
                    break
                if it == maxit:
                    status = ST_OK
                    break
            else:
                if rr <= tol:
                    status = ST_OK
                    break
                verdict = _stop_rule(hist)
                if verdict is not None:
                    status = verdict
                    break
                if it == maxit:
                    break
            x = x + correction(r)
            steps += 1
    xout = (x if status == ST_OK else best[1]) * (2.0 ** k)
    out = {"X": xout, "steps": steps, "hist": hist, "status": status}
    if iterates:
        out["iterates"] = seq
    return out


# ---------------------------------------------------------------------------
# Sylvester and adjoint solves


def trsyl(s, st, c, single=False):
    """S Y + Y St = C, S and St upper triangular (complex), back-substitution."""
    dt = np.complex64 if single else np.complex128
    ct = ctypes.c_float if single else ctypes.c_double
    s, st, c = _f(s, dt), _f(st, dt), _f(c, dt)
    m, n = c.shape
    y = np.zeros((m, n), dtype=dt, order="F")
    fn = lib().orc_trsyl_c if single else lib().orc_trsyl_z
    fn(m, n, _ptr(s, ct), _ptr(st, ct), _ptr(c, ct), _ptr(y, ct))
    return y


def rtrsyl(s, st, c, blks=32, single=False):
    """Alg. 1 block recursion for S Y + Y St = C."""
    dt = np.complex64 if single else np.complex128
    ct = ctypes.c_float if single else ctypes.c_double
    s, st = _f(s, dt), _f(st, dt)
    y = _f(c, dt).copy(order="F")
    m, n = y.shape
    fn = lib().orc_rtrsyl_c if single else lib().orc_rtrsyl_z
    fn(m, n, _ptr(s, ct), _ptr(st, ct), _ptr(y, ct), int(blks))
    return y


def real_schur(a, single=False):
    """Real Schur form A = Q T Q^T (remark in Sec. 2.2.1): T quasi-upper-
    triangular with 1x1 blocks and standardised 2x2 blocks (equal diagonal
    entries, off-diagonal entries of opposite sign) for complex conjugate
    eigenvalue pairs.  The decomposition is the LAPACK routine behind
    scipy.linalg.schur (a library step; float32 input stays in single
    precision).  Returns (T, Q)."""
    import scipy.linalg
    dt = np.float32 if single else np.float64
    t, q = scipy.linalg.schur(np.asarray(a, dtype=dt), output="real")
    return np.asfortranarray(t), np.asfortranarray(q)


def sqrt_2x2(b):
    """Principal square root of a real 2x2 block by the Cayley-Hamilton
    closed form X = (B + d I) / t, d = det(B)^1/2, t = (tr B + 2 d)^1/2."""
    b = _f(b, np.float64)
    x = np.zeros((2, 2), order="F")
    _check(lib().orc_sqrt_2x2_d(_ptr(b, ctypes.c_double), _ptr(x, ctypes.c_double)), "sqrt_2x2")
    return x


def trsqrt_quasi(t, single=False):
    """Square root of a quasi-upper-triangular T by blocks (Eq. (subst) with
    1x1 / 2x2 diagonal blocks as units)."""
    dt = np.float32 if single else np.float64
    ct = ctypes.c_float if single else ctypes.c_double
    t = _f(t, dt)
    n = t.shape[0]
    u = np.zeros((n, n), dtype=dt, order="F")
    fn = lib().orc_trsqrt_quasi_s if single else lib().orc_trsqrt_quasi_d
    _check(fn(n, _ptr(t, ct), _ptr(u, ct)), "trsqrt_quasi")
    return u


def trsyl_quasi(s, st, c):
    """S Y + Y St = C with quasi-upper-triangular S, St (float64), block
    back-substitution."""
    s, st, c = _f(s, np.float64), _f(st, np.float64), _f(c, np.float64)
    m, n = c.shape
    y = np.zeros((m, n), order="F")
    dp = ctypes.c_double
    lib().orc_trsyl_quasi_d(m, n, _ptr(s, dp), _ptr(st, dp), _ptr(c, dp), _ptr(y, dp))
    return y


def rtrsyl_quasi(s, st, c, blks=32, single=False):
    """Alg. 1 for quasi-upper-triangular S, St: splits never cut a 2x2 block."""
    dt = np.float32 if single else np.float64
    ct = ctypes.c_float if single else ctypes.c_double
    s, st = _f(s, dt), _f(st, dt)
    y = _f(c, dt).copy(order="F")
    m, n = y.shape
    fn = lib().orc_rtrsyl_quasi_s if single else lib().orc_rtrsyl_quasi_d
    fn(m, n, _ptr(s, ct), _ptr(st, ct), _ptr(y, ct), int(blks))
    return y


def sqrtm_real(a, return_factors=False):
    """Principal square root of a real matrix by the real Schur route in
    float64: A = Q T Q^T, U = T^{1/2} (quasi-triangular), X = Q U Q^T."""
    a = _f(a, np.float64)
    if a.shape[0] == 0:
        x = np.zeros((0, 0))
        return (x, None) if return_factors else x
    if not np.all(np.isfinite(a)):
        raise OracleError("sqrtm_real: non-finite input")
    t, q = real_schur(a)
    u = trsqrt_quasi(t)
    x = np.asfortranarray(q @ u @ q.T)
    if return_factors:
        return x, {"Q": q, "T": t, "U": u}
    return x


def kron_sylvester(s, st, c):
    """Brute force: (I kron S + St^T kron I) vec(Y) = vec(C) (Sec. 3.1 vec form)."""
    s = np.asarray(s, dtype=np.complex128)
    st = np.asarray(st, dtype=np.complex128)
    c = np.asarray(c, dtype=np.complex128)
    m, n = c.shape
    big = np.kron(np.eye(n), s) + np.kron(st.T, np.eye(m))
    y = np.linalg.solve(big, c.reshape(-1, order="F"))
    return y.reshape((m, n), order="F")


def adjoint(x, gbar):
    """G with X^H G + G X^H = Gbar (complex128), through the Schur form of X.
    Real inputs give a real G."""
    is_real = not (np.iscomplexobj(x) or np.iscomplexobj(gbar))
    xz = _f(x, np.complex128)
    gz = _f(gbar, np.complex128)
    n = xz.shape[0]
    g = np.zeros((n, n), dtype=np.complex128, order="F")
    dp = ctypes.c_double
    _check(lib().orc_adjoint_z(n, _ptr(xz, dp), _ptr(gz, dp), _ptr(g, dp)), "adjoint")
    return np.asfortranarray(g.real) if is_real else g


def adjoint_spd(q, lam, gbar):
    """Closed form of the adjoint for X = Q diag(lam^1/2) Q^T (SPD): in the
    eigenbasis X G + G X = Gbar is diagonal, g_ij = (Q^T Gbar Q)_ij /
    (lam_i^1/2 + lam_j^1/2)."""
    s = np.sqrt(np.asarray(lam, dtype=np.float64))
    q = np.asarray(q, dtype=np.float64)
    h = (q.T @ np.asarray(gbar, dtype=np.float64) @ q) / (s[:, None] + s[None, :])
    return q @ h @ q.T


def kron_adjoint(x, gbar):
    """Brute force for X^H G + G X^H = Gbar: (I kron X^H + conj(X) kron I) vec G."""
    x = np.asarray(x, dtype=np.complex128)
    n = x.shape[0]
    xh = x.conj().T
    big = np.kron(np.eye(n), xh) + np.kron(xh.T, np.eye(n))
    g = np.linalg.solve(big, np.asarray(gbar, dtype=np.complex128).reshape(-1, order="F"))
    return g.reshape((n, n), order="F")


# ---------------------------------------------------------------------------
# Accuracy measures (Sec. 5.1)


def relres(x, a):
    """||X^2 - A||_F / ||A||_F."""
    return float(np.linalg.norm(x @ x - a) / np.linalg.norm(a))


def relerr(x, xref):
    """||X - Xref||_F / ||Xref||_F."""
    return float(np.linalg.norm(x - xref) / np.linalg.norm(xref))


# ---------------------------------------------------------------------------
# Mixed-precision emulator (Alg. 2 / Alg. 3)

ST_OK, ST_NOT_CONVERGED, ST_DIVERGED, ST_NO_PRINCIPAL, ST_NONFINITE = (
    "ok", "not_converged", "diverged", "no_principal", "nonfinite")


def scale_exponent(a):
    """k with A/4^k of Frobenius norm near sqrt(n) (exact power-of-4 scaling
    before the down-conversion, Sec. 5)."""
    n = a.shape[0]
    nrm = np.linalg.norm(a)
    if nrm == 0 or n == 0:
        return 0
    return int(np.round(np.log(nrm / np.sqrt(n)) / np.log(4.0)))


def _stop_rule(hist):
    """Divergence and stagnation reading of the paper's 'diverges in our
    tests' (Sec. 5.1), applied after each new residual:
      diverged   if the residual is non-finite, grew on two consecutive
                 sweeps, or exceeds 10x the first residual;
      stagnated  if it failed to drop below 0.9x the previous residual on two
                 consecutive sweeps."""
    r = hist[-1]
    if not np.isfinite(r):
        return ST_DIVERGED
    if r > 10.0 * hist[0]:
        return ST_DIVERGED
    if len(hist) >= 3 and hist[-1] > hist[-2] and hist[-2] > hist[-3]:
        return ST_DIVERGED
    if len(hist) >= 3 and hist[-1] > 0.9 * hist[-2] and hist[-2] > 0.9 * hist[-3]:
        return ST_NOT_CONVERGED
    return None


def emulate_mixed(a, structure="auto", low="fp32", maxit=30, tol=1e-13, blks=32,
                  factor=None, x0=None, iterates=False, schur_form="complex"):
    """Alg. 3 (SPD, structure='spd') or Alg. 2 (structure='general') with the
    low precision emulated by this module's single-precision factorisation and
    float32 arithmetic for the transforms, float64 for residual and update.

    factor: optional SPD factor {"Q": q, "s": s} used instead of the
      emulator's own factorisation (the frozen Z = Q diag(s) Q^T of the
      convergence theorem); it belongs to A itself (no scaling), and low
      ("fp32" or "fp64") is the arithmetic of its transforms.
    x0: optional start (float64) instead of X_0 = Q diag(s) Q^T; only with
      `factor`.
    iterates: also return the list of iterates X_0, X_1, ... (unscaled).
    schur_form: "complex" (Alg. 2 as printed) or "real" (real input only: the
      real Schur form and the quasi-triangular solves of the remark in
      Sec. 2.2.1).
    tol < 0 nullifies the stopping test (the accuracy experiments of Sec. 5.1):
      exactly maxit corrections, status ok, X the last iterate.

    Returns dict(X, steps, hist, status[, iterates]).  steps counts applied
    corrections; hist holds ||R_k||_F / ||A||_F for every residual evaluated.
    On a failure X is the iterate with the smallest residual.
    """
    a = np.asarray(a)
    n = a.shape[0]
    is_real = not np.iscomplexobj(a)
    if structure == "auto":
        structure = "spd" if (is_real and np.array_equal(a, a.T)) else "general"
    if not np.all(np.isfinite(a)):
        return {"X": None, "steps": 0, "hist": [], "status": ST_NONFINITE}
    if x0 is not None and factor is None:
        raise ValueError("x0 needs an explicit factor")
    lowt = np.float32 if low == "fp32" else np.float64
    k = 0 if factor is not None else scale_exponent(a)
    asc = a / (4.0 ** k)
    na = np.linalg.norm(asc)
    if structure == "spd":
        if factor is not None:
            q = np.asarray(factor["Q"], dtype=lowt)
            s = np.asarray(factor["s"], dtype=lowt)
        else:
            lam, q = syev(asc.astype(np.float32), single=True)
            if np.any(lam <= 0):
                return {"X": None, "steps": 0, "hist": [], "status": ST_NO_PRINCIPAL}
            s = np.sqrt(lam).astype(np.float32)
        x = ((q * s[None, :]) @ q.T).astype(np.float64) if x0 is None else np.array(x0, np.float64)
        denom = (s[:, None] + s[None, :]).astype(lowt)

        def correction(r):
            rl = r.astype(lowt)
            rt = q.T @ rl @ q
            y = rt / denom
            return (q @ y @ q.T).astype(np.float64)
    elif schur_form == "real":
        if factor is not None or not is_real:
            raise ValueError("the real Schur route takes real input and its own factor")
        single = low == "fp32"
        t, q = real_schur(asc, single=single)
        try:
            u = trsqrt_quasi(t, single=single)
        except OracleError:
            return {"X": None, "steps": 0, "hist": [], "status": ST_NO_PRINCIPAL}
        x = (q @ u @ q.T).astype(np.float64)

        def correction(r):
            rl = r.astype(lowt)
            rt = q.T @ rl @ q
            y = rtrsyl_quasi(u, u, rt, blks=blks, single=single)
            return (q @ y @ q.T).astype(np.float64)
    else:
        if factor is not None:
            raise ValueError("an explicit factor is supported for the SPD route only")
        t, q = schur(asc.astype(np.complex64), single=True)
        d = np.diag(t)
        if np.any((d.imag == 0) & (d.real <= 0)):
            return {"X": None, "steps": 0, "hist": [], "status": ST_NO_PRINCIPAL}
        s = trsqrt(t, single=True)
        qh = q.conj().T
        x0c = (q @ s @ qh).astype(np.complex128)
        x = x0c.real.copy() if is_real else x0c

        def correction(r):
            rl = r.astype(np.complex64)
            rt = qh @ rl @ q
            y = rtrsyl(s, s, rt, blks=blks, single=True)
            dx = (q @ y @ qh).astype(np.complex128)
            return dx.real if is_real else dx

    hist = []
    seq = []
    best = (np.inf, x)
    status = ST_NOT_CONVERGED
    steps = 0
    with np.errstate(over="ignore", invalid="ignore"):
        for it in range(maxit + 1):
            if iterates:
                seq.append(x * (2.0 ** k))
            r = asc - x @ x
            rr = float(np.linalg.norm(r) / na)
            hist.append(rr)
            if rr < best[0]:
                best = (rr, x)
            if tol < 0:
                # nullified stopping test (Sec. 5.1 accuracy experiments):
                # exactly maxit corrections, the last iterate is kept
                if not np.isfinite(rr):
                    status = ST_DIVERGED
                    break
                if it == maxit:
                    status = ST_OK
                    break
            else:
                if rr <= tol:
                    status = ST_OK
                    break
                verdict = _stop_rule(hist)
                if verdict is not None:
                    status = verdict
                    break
                if it == maxit:
                    break
            x = x + correction(r)
            steps += 1
    xout = (x if status == ST_OK else best[1]) * (2.0 ** k)
    out = {"X": xout, "steps": steps, "hist": hist, "status": status}
    if iterates:
        out["iterates"] = seq
    return out
